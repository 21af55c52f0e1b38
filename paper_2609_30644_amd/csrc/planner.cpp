// MR. POP planner driver (Alg. 1) and the search-primitive entry points.
//
// The driver keeps every roadmap and both search trees on the device and
// runs the search in bulk-synchronous rounds of P candidates:
//   sample -> NEAREST in the extended tree -> dRRT oracle -> validate the
//   extensions -> insert in candidate order -> NEAREST in the other tree ->
//   validate the connections -> pick the cheapest connection.
// Sampling with the first NEAREST, and insertion with the second NEAREST and
// the connection edges, run as one launch each (one workgroup per candidate).
// One small status record per round comes back to the host: the selection
// kernel writes it straight into pinned memory.  The host decides whether
// the search ended, swaps the trees when the extended one has grown larger,
// and extracts a path on success.
//
// The driver is a PlanJob: its device work goes through an Exec, which runs
// it at once on a stream for mrpop_plan, or merges it with other instances'
// work for mrpop_plan_batch.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "plan_job.h"

using namespace mrpop;

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// One arm alone with the environment (for single-arm roadmap checks).
mrpop_status arm_scene(mrpop_ctx *ctx, const mrpop_scene *sc, int r, mrpop_scene **out) {
  const HostRobot &h = sc->h_robots[r];
  mrpop_robot rb{h.n_joints, h.dh.data(), h.q_lo.data(), h.q_hi.data(), h.base.data(),
                 (int32_t)h.link.size(), h.link.data(), h.xyzr.data()};
  mrpop_env env{(int32_t)(sc->h_env_s.size() / 4), sc->h_env_s.empty() ? nullptr : sc->h_env_s.data(),
                (int32_t)(sc->h_env_b.size() / 6), sc->h_env_b.empty() ? nullptr : sc->h_env_b.data()};
  return mrpop_scene_create(ctx, &rb, 1, &env, out);
}

// Sub-allocations of one device allocation (256-byte aligned).
struct ArenaPlan {
  std::vector<std::pair<void **, size_t>> items;
  template <class T>
  void add(T **p, size_t n) {
    items.push_back({(void **)p, std::max<size_t>(n, 1) * sizeof(T)});
  }
  size_t total() const {
    size_t t = 0;
    for (auto &it : items) t += (it.second + 255) & ~size_t(255);
    return t;
  }
  void assign(void *base) {
    size_t off = 0;
    for (auto &it : items) {
      *it.first = (unsigned char *)base + off;
      off += (it.second + 255) & ~size_t(255);
    }
  }
};

}  // namespace

namespace mrpop {

// Device work launched at once on one stream.  Consecutive validations are
// held back and launched together (one many-scene launch) when the next
// other command arrives or at sync(): they are independent by contract.
class PlainExec : public Exec {
  static constexpr int64_t kKernelCopyMax = 4096;

 public:
  PlainExec(mrpop_ctx *ctx, hipStream_t s) : ctx_(ctx), s_(s) {}
  ~PlainExec() override {
    for (void *p : staging_) (void)hipHostFree(p);
  }
  hipError_t submit(const Cmd &c) override {
    if (c.op == Op::Validate) {
      if (c.val.n > 0) val_.push_back(c.val);
      return hipSuccess;
    }
    hipError_t e = flush_validations();
    if (e != hipSuccess) return e;
    // small copies (round status, counts) by the library's copy kernel, which
    // starts as soon as the previous kernel ends; large ones by the runtime
    if (c.op == Op::Copy && c.copy.bytes > kKernelCopyMax)
      return hipMemcpyAsync(c.copy.dst, c.copy.src, c.copy.bytes, hipMemcpyDefault, s_);
    return launch_op(c.op, c.args(), s_);
  }
  // Each run of one kind launches as one kernel, kGroupMax records at a time;
  // copies too large for the copy kernel go to the runtime one by one.
  hipError_t submit_independent(const Cmd *cs, int n) override {
    hipError_t e = flush_validations();
    if (e != hipSuccess) return e;
    for (int i = 0; i < n;) {
      const Op op = cs[i].op;
      if (op == Op::Validate) return hipErrorInvalidValue;
      if (op == Op::Copy && cs[i].copy.bytes > kKernelCopyMax) {
        if ((e = submit(cs[i])) != hipSuccess) return e;
        ++i;
        continue;
      }
      const void *recs[kGroupMax];
      int k = 0;
      while (i < n && k < kGroupMax && cs[i].op == op && !(op == Op::Copy && cs[i].copy.bytes > kKernelCopyMax))
        recs[k++] = cs[i++].args();
      if ((e = launch_op_group(op, recs, k, s_)) != hipSuccess) return e;
    }
    return hipSuccess;
  }
  // Spins on the flag: the round trip is about half that of a stream
  // synchronisation.  The stream is polled now and then, so that a failed
  // kernel is reported instead of waited for.
  hipError_t wait_flag(const uint32_t *flag, uint32_t value) override {
    hipError_t e = flush_validations();
    if (e != hipSuccess) return e;
    for (uint32_t k = 1;; ++k) {
      if (__atomic_load_n(flag, __ATOMIC_ACQUIRE) == value) break;
      if ((k & 1023u) == 0) {
        e = hipStreamQuery(s_);
        if (e == hipSuccess) {  // all work done: the flag must be there now
          if (__atomic_load_n(flag, __ATOMIC_ACQUIRE) == value) break;
          return hipErrorUnknown;
        }
        if (e != hipErrorNotReady) return e;
      }
    }
    used_ = 0;  // everything before the flag's writer has completed
    return hipSuccess;
  }
  hipError_t sync() override {
    hipError_t e = flush_validations();
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s_);
    used_ = 0;  // every staged upload has completed
    return e;
  }

 private:
  hipError_t flush_validations() {
    if (val_.empty()) return hipSuccess;
    std::vector<ValidateReq> v;
    v.swap(val_);
    if (v.size() == 1) {
      const ValidateReq &q = v[0];
      void *base = nullptr;
      if (scratch_slot(ctx_, 1, validate_scratch_bytes(q.n), &base) != MRPOP_OK) return hipErrorOutOfMemory;
      ValidateScratch ws = validate_scratch_layout(base, q.n);
      ws.counters = q.counters;
      if (q.n_codes && q.n <= kFusedMaxEdges) {  // counts made by the producer: one launch
        uint32_t *arrived = nullptr, *flags = nullptr, token = 0;
        const hipError_t e = small_launch_state(ctx_, &arrived, &flags, &token);
        if (e != hipSuccess) return e;
        ws.flags = flags;
        return launch_validate_small(*q.scene, q.qa, q.qb, q.n, q.n_codes, q.out, ws, arrived, token, s_,
                                     profile_slot(ctx_), ctx_->profiling ? ctx_->prof_totals : nullptr,
                                     &ctx_->last_grid, &ctx_->last_block);
      }
      return launch_validate(*q.scene, q.qa, q.qb, q.n, q.res, nullptr, q.out, ws, s_, profile_slot(ctx_),
                             ctx_->profiling ? ctx_->prof_totals : nullptr, &ctx_->last_grid, &ctx_->last_block);
    }
    int r_max = 1, dof_max = 1;
    int64_t flat = 0;
    for (const ValidateReq &q : v) {
      r_max = std::max(r_max, (int)q.scene->n_robots);
      dof_max = std::max(dof_max, (int)q.scene->dof);
      flat += q.n;
    }
    int W = 0, cache = 0;
    seg_shape(r_max, flat, &W, &cache);
    const size_t bytes = sizeof(ValSeg) * v.size();
    const bool small = (int)v.size() <= kSegSmallMax && small_scan(flat, dof_max);
    hipError_t e;
    if (small) {  // the table travels as kernel arguments
      ValSeg h[kSegSmallMax];
      int64_t e0 = 0;
      for (size_t i = 0; i < v.size(); ++i) {
        fill_seg(h[i], v[i], e0, W);
        e0 += v[i].n;
      }
      if ((e = ensure_seg_buffers(bytes, flat)) != hipSuccess) return e;
      return launch_validate_segments_small(h, (int)v.size(), r_max, flat, (ValSeg *)d_segs_,
                                            seg_scratch_layout(seg_ws_, flat), s_, profile_slot(ctx_),
                                            ctx_->profiling ? ctx_->prof_totals : nullptr, &ctx_->last_grid,
                                            &ctx_->last_block);
    }
    if (used_ == staging_.size() || stage_bytes_ < bytes) {
      if (stage_bytes_ < bytes) {  // all staging buffers grow together (only between syncs if in use)
        if (used_ > 0 && (e = hipStreamSynchronize(s_)) != hipSuccess) return e;
        for (void *p : staging_) (void)hipHostFree(p);
        staging_.clear();
        used_ = 0;
        stage_bytes_ = std::max(bytes, 2 * stage_bytes_);
      }
      void *p = nullptr;
      if ((e = hipHostMalloc(&p, stage_bytes_)) != hipSuccess) return e;
      staging_.push_back(p);
    }
    ValSeg *h = (ValSeg *)staging_[used_++];
    int64_t e0 = 0;
    for (size_t i = 0; i < v.size(); ++i) {
      fill_seg(h[i], v[i], e0, W);
      e0 += v[i].n;
    }
    if ((e = ensure_seg_buffers(bytes, flat)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(d_segs_, h, bytes, hipMemcpyHostToDevice, s_)) != hipSuccess) return e;
    return launch_validate_segments((ValSeg *)d_segs_, (int)v.size(), r_max, flat, seg_scratch_layout(seg_ws_, flat),
                                    s_, profile_slot(ctx_), ctx_->profiling ? ctx_->prof_totals : nullptr,
                                    &ctx_->last_grid, &ctx_->last_block);
  }

  static void fill_seg(ValSeg &g, const ValidateReq &q, int64_t edge0, int W) {
    std::memset(&g, 0, sizeof(g));
    g.sc = *q.scene;
    g.qa = q.qa;
    g.qb = q.qb;
    g.edge0 = edge0;
    g.n_edges = q.n;
    g.res = q.res;
    g.S = seg_link_split(q.scene->n_robots, W);
    g.out = q.out;
    g.counters = q.counters;
  }
  // Device segment table (bytes) and scratch for n_flat edges, in the
  // context's scratch slots 2 and 3 (kept across plans, so that a plan does
  // not allocate them again); a buffer in use by queued work is only
  // replaced after the stream has drained.
  hipError_t ensure_seg_buffers(size_t bytes, int64_t flat) {
    const size_t ws_bytes = seg_scratch_bytes(flat);
    if (ctx_->scratch[2].bytes < bytes || ctx_->scratch[3].bytes < ws_bytes) {
      const hipError_t e = hipStreamSynchronize(s_);
      if (e != hipSuccess) return e;
    }
    if (scratch_slot(ctx_, 2, bytes, &d_segs_) != MRPOP_OK) return hipErrorOutOfMemory;
    if (scratch_slot(ctx_, 3, ws_bytes, &seg_ws_) != MRPOP_OK) return hipErrorOutOfMemory;
    return hipSuccess;
  }

  mrpop_ctx *ctx_;
  hipStream_t s_;
  std::vector<ValidateReq> val_;
  std::vector<void *> staging_;  // pinned uploads of segment tables, free again after sync()
  size_t used_ = 0, stage_bytes_ = 0;
  void *d_segs_ = nullptr, *seg_ws_ = nullptr;  // the context's scratch slots 2 and 3
};

PlanJob::~PlanJob() {
  // the blocks go back to the pool only once no queued work uses them: run()
  // ends with a synchronisation; a run that returned early is waited for here
  if (!synced_ && (arena_ || host_block_)) (void)hipDeviceSynchronize();
  if (arena_) pool_free(ctx_, false, arena_, arena_got_);
  if (host_block_) pool_free(ctx_, true, host_block_, host_got_);
  if (pin_path_) (void)hipHostFree(pin_path_);
}

double PlanJob::elapsed_() const { return now_s() - t_start_; }
bool PlanJob::out_of_time_() const { return P_.time_budget_s > 0 && elapsed_() >= P_.time_budget_s; }

void PlanJob::set_sizes_(const mrpop_scene *scene, const mrpop_plan_params &P) {
  R_ = scene->n_robots;
  D_ = scene->dof;
  PC_ = P.candidates;
  rm_cap_ = P.direct ? 4 : P.max_roadmap_nodes;  // direct mode keeps no roadmaps
  edge_cap_ = rm_cap_ * 32;
  col_cap_ = 2 * edge_cap_;
  cand_batch_ = 4 * P.n_roadmap;
  pair_cap_ = P.n_roadmap * rm_cap_;
  tcap_ = P.max_tree_nodes;
  batch_rows_ = (int64_t)(2 + (P.rewire ? kRwSlots : 0)) * PC_;
  path_max_ = 16384;
  max_nj_ = 0;
  for (int r = 0; r < R_; ++r) max_nj_ = std::max(max_nj_, scene->nj[r]);
}

size_t PlanJob::plan_arena_(void *base) {
  const int R = R_, D = D_, PC = PC_, max_nj = max_nj_;
  ArenaPlan ar;
  ar.add(&qs_, D);
  ar.add(&qg_, D);
  ar.add(&rm_V_, (size_t)R * rm_cap_ * kRmStride);
  ar.add(&rm_rowptr_, (size_t)R * (rm_cap_ + 1));
  ar.add(&rm_col_, (size_t)R * col_cap_);
  ar.add(&rm_edges_, (size_t)R * edge_cap_ * 2);
  ar.add(&rm_nv_, R);
  ar.add(&rm_ne_, R);
  ar.add(&cand_, (size_t)R * cand_batch_ * kRmStride);
  ar.add(&cand_valid_, (size_t)R * cand_batch_);
  ar.add(&cand_codes_, (size_t)R * cand_batch_);
  ar.add(&pair_ids_, (size_t)pair_cap_ * 2);
  ar.add(&pair_qa_, (size_t)pair_cap_ * max_nj);
  ar.add(&pair_qb_, (size_t)pair_cap_ * max_nj);
  ar.add(&pair_valid_, pair_cap_);
  ar.add(&pair_codes_, pair_cap_);
  ar.add(&rm_i_, (size_t)R * kRmInts);
  ar.add(&uf_, (size_t)R * rm_cap_);
  ar.add(&deg_, (size_t)R * rm_cap_);
  for (int t = 0; t < 2; ++t) {
    ar.add(&tq_[t], (size_t)D * tcap_);
    ar.add(&tg_[t], tcap_);
    ar.add(&tvid_[t], (size_t)R * tcap_);
    ar.add(&tpar_[t], tcap_);
    ar.add(&tn_[t], 1);
  }
  if (P_.rewire) {
    for (int t = 0; t < 2; ++t) ar.add(&te_[t], tcap_);
    ar.add(&prop_z_, (size_t)kRwSlots * PC);
    ar.add(&prop_cost_, (size_t)kRwSlots * PC);
    ar.add(&prop_len_, (size_t)kRwSlots * PC);
    ar.add(&e_new_, PC);
    ar.add(&rw_key_, tcap_);
  }
  ar.add(&q_rand_, (size_t)PC * D);
  ar.add(&c_rand_, PC);
  ar.add(&near_idx_, PC);
  ar.add(&q_new_, (size_t)PC * D);
  ar.add(&g_new_, PC);
  ar.add(&vid_new_, (size_t)R * PC);
  ar.add(&alive_, PC);
  // a round's edge batch: extension edges in rows [0, PC), connection edges
  // in rows [PC, 2 PC), with rewiring the proposal edges after them; their
  // bits and state-count codes alike
  ar.add(&ea_, (size_t)batch_rows_ * D);
  ar.add(&eb_, (size_t)batch_rows_ * D);
  ar.add(&valid_, (size_t)batch_rows_);
  ar.add(&ins_idx_, PC);
  ar.add(&budget_, PC);
  ar.add(&conn_idx_, PC);
  ar.add(&codes_ext_, (size_t)batch_rows_);
  ar.add(&cnt_, (size_t)(2 + R) * 16);
  ar.add(&status_, 1);
  ar.add(&ss_, 1);
  ar.add(&path_d_, (size_t)path_max_ * D);
  ar.add(&path_vid_d_, (size_t)path_max_ * R);
  ar.add(&d_nj_, R);
  ar.add(&d_qoff_, R);
  if (base) ar.assign(base);
  return ar.total();
}

size_t PlanJob::device_bytes_for(const mrpop_scene *scene, const mrpop_plan_params &params) {
  PlanJob j;
  j.P_ = params;
  j.set_sizes_(scene, params);
  return j.plan_arena_(nullptr) + (params.direct ? 0 : (size_t)scene->n_robots * scene->blob_bytes);
}

mrpop_status PlanJob::prepare(mrpop_ctx *ctx, const mrpop_scene *scene, const float *q_start, const float *q_goal,
                              const mrpop_plan_params &P) {
  ctx_ = ctx;
  scene_ = scene;
  P_ = P;
  if (P.candidates < 1 || P.candidates > kMaxCandidates || !(P.resolution > 0.f) || !std::isfinite(P.resolution) ||
      P.max_rounds < 1 || P.max_iterations < 1 || P.max_growth_rounds < 1 || P.n_roadmap < 1 ||
      P.max_tree_nodes < 2 || P.max_roadmap_nodes < 4 || P.max_roadmap_nodes > kUfMaxVertices ||
      !(P.delta > 0.f) || P.time_budget_s < 0 || std::isnan(P.warm_cost) || (P.direct != 0 && P.direct != 1) ||
      (P.direct && !(P.step > 0.f && std::isfinite(P.step))) || (P.rewire != 0 && P.rewire != 1) ||
      (P.rewire && (P.direct || P.max_roadmap_nodes > kRwMaxRoadmap)))
    return fail_(MRPOP_E_INVALID_ARG, "plan: parameter out of range");
  R_ = scene->n_robots;
  D_ = scene->dof;
  PC_ = P.candidates;
  for (int j = 0; j < D_; ++j)
    if (!std::isfinite(q_start[j]) || !std::isfinite(q_goal[j]))
      return fail_(MRPOP_E_NONFINITE, "plan: non-finite start or goal");
  std::memset(&st_, 0, sizeof(st_));
  st_.time_to_first_s = -1.0;
  st_.first_round = -1;
  c_best_ = P.warm_cost;

  set_sizes_(scene, P);
  const int R = R_, D = D_;
  const size_t arena_bytes = plan_arena_(nullptr);
  hipError_t e = hipSetDevice(ctx->device);
  if (e == hipSuccess) e = pool_alloc(ctx, false, arena_bytes, &arena_, &arena_got_);
  if (e != hipSuccess) {
    arena_ = nullptr;
    return e == hipErrorOutOfMemory ? fail_(MRPOP_E_NOMEM, "plan: device memory") : hip_fail_(e, "hipMalloc(plan)");
  }
  plan_arena_(arena_);
  ca_ = ea_ + (size_t)PC_ * D_;
  cb_ = eb_ + (size_t)PC_ * D_;
  cvalid_ = valid_ + PC_;
  codes_conn_ = codes_ext_ + PC_;
  device_bytes_ = arena_bytes;
  // the small pinned buffers share one block (256-byte aligned parts)
  const size_t up_floats = 2 * (size_t)D + (size_t)R * 2 * kRmStride;
  ArenaPlan hp;
  hp.add(&pin_, 1);
  hp.add(&pin_rm_, (size_t)R * (kRmInts + 1));
  hp.add(&pin_cnt_, (size_t)R * 16);
  hp.add(&upload_, up_floats);
  hp.add(&upload_i_, 4 * (size_t)R + 4);
  if ((e = pool_alloc(ctx, true, hp.total(), &host_block_, &host_got_)) != hipSuccess) {
    host_block_ = nullptr;
    return hip_fail_(e, "hipHostMalloc");
  }
  hp.assign(host_block_);
  std::memset(pin_, 0, sizeof(Pinned));  // round numbers start at 1, so no stale record matches

  h_qoff_.assign(R, 0);
  h_nj_.assign(R, 0);
  for (int r = 0, o = 0; r < R; ++r) {
    h_qoff_[r] = o;
    h_nj_[r] = scene->nj[r];
    o += scene->nj[r];
  }
  // uploads: start, goal, roadmap seeds (vertex 0 = the arm's start, 1 = its goal)
  std::memcpy(upload_, q_start, sizeof(float) * D);
  std::memcpy(upload_ + D, q_goal, sizeof(float) * D);
  float *init = upload_ + 2 * D;
  std::fill(init, init + (size_t)R * 2 * kRmStride, 0.f);
  for (int r = 0; r < R; ++r)
    for (int j = 0; j < h_nj_[r]; ++j) {
      init[((size_t)r * 2 + 0) * kRmStride + j] = q_start[h_qoff_[r] + j];
      init[((size_t)r * 2 + 1) * kRmStride + j] = q_goal[h_qoff_[r] + j];
    }
  for (int r = 0; r < R; ++r) {
    upload_i_[r] = h_nj_[r];
    upload_i_[R + r] = h_qoff_[r];
    upload_i_[2 * R + r] = 2;  // roadmap vertex counts
    upload_i_[3 * R + r] = 0;  // roadmap edge counts
  }
  upload_i_[4 * R] = 0;  // union-find parents of vertices 0 and 1
  upload_i_[4 * R + 1] = 1;
  arms_.assign(R, nullptr);
  if (!P.direct && (int)scene->arm_cache.size() != R) {  // one-arm scenes of the roadmaps, once per scene
    std::vector<mrpop_scene *> built(R, nullptr);
    for (int r = 0; r < R; ++r) {
      mrpop_status a = arm_scene(ctx, scene, r, &built[r]);
      if (a != MRPOP_OK) {
        for (mrpop_scene *b : built) mrpop_scene_destroy(b);
        return fail_(a, "plan: arm scene: " + ctx->last_error);
      }
    }
    for (mrpop_scene *old : scene->arm_cache) mrpop_scene_destroy(old);
    scene->arm_cache = built;
  }
  for (int r = 0; r < R && !P.direct; ++r) {
    arms_[r] = scene->arm_cache[r];
    device_bytes_ += arms_[r]->blob_bytes;
  }
  rm_n_.assign(R, 2);
  return MRPOP_OK;
}

mrpop_status PlanJob::copy_(Exec &ex, void *dst, const void *src, size_t bytes) {
  Cmd c;
  c.op = Op::Copy;
  c.copy = CopyArgs{dst, src, (int64_t)bytes};
  const hipError_t e = ex.submit(c);
  return e == hipSuccess ? MRPOP_OK : hip_fail_(e, "copy");
}

mrpop_status PlanJob::group_(Exec &ex, std::vector<Cmd> &cs) {
  const hipError_t e = cs.empty() ? hipSuccess : ex.submit_independent(cs.data(), (int)cs.size());
  cs.clear();
  return e == hipSuccess ? MRPOP_OK : hip_fail_(e, "group");
}

mrpop_status PlanJob::validate_(Exec &ex, const mrpop_scene *sc, const float *a, const float *b, int64_t n,
                                float res, uint8_t *out, uint64_t *counters, const int32_t *n_codes) {
  if (n <= 0) {
    Cmd z;
    z.op = Op::Fill;
    z.fill = FillArgs{(uint32_t *)counters, 0u, 32};
    const hipError_t e = ex.submit(z);
    return e == hipSuccess ? MRPOP_OK : hip_fail_(e, "fill");
  }
  Cmd c;
  c.op = Op::Validate;
  c.val = ValidateReq{&sc->dev, a, b, n, res, out, counters, n_codes};
  const hipError_t e = ex.submit(c);
  return e == hipSuccess ? MRPOP_OK : hip_fail_(e, "validate launch");
}

// (inside the coroutines run() and roadmap_())
#define SUBMIT(OPV, FIELD, ...)                            \
  do {                                                     \
    Cmd c_;                                                \
    c_.op = OPV;                                           \
    c_.FIELD = __VA_ARGS__;                                \
    const hipError_t e_ = ex.submit(c_);                   \
    if (e_ != hipSuccess) co_return hip_fail_(e_, #FIELD); \
  } while (0)

#define SYNC()                                             \
  do {                                                     \
    const hipError_t e_ = co_await SyncPoint{ex};          \
    if (e_ != hipSuccess) co_return hip_fail_(e_, "sync"); \
  } while (0)

#define TRY(expr)                     \
  do {                                \
    const mrpop_status s_ = (expr);   \
    if (s_ != MRPOP_OK) co_return s_; \
  } while (0)

// ROADMAP (Alg. 2) for outer iteration `it`.  Every arm still unconnected
// grows in the same steps (the arms' commands of a step submitted as one
// independent group): free samples, counts of candidate pairs (new vertex,
// any vertex within delta), then the pairs themselves, their single-arm
// validation and the union of the components they join; connectivity of
// start and goal is read from the union-find.  A growth round takes one host
// round trip: the next round's first sampling pass is queued behind the
// union before the host has read which arms it connected (an arm it
// connected draws and accepts nothing, by a flag the union sets on the
// device), and one wait returns both.  Further passes (when a batch of
// samples held too few free ones) take a round trip each.  The adjacency used
// by the extension oracle is rebuilt once at the end.
mrpop_status PlanJob::rm_pass_(Exec &ex, int it, int g, int64_t j0, const std::vector<int> &act,
                               const std::vector<int> &counted, bool speculative, const std::vector<int> &need,
                               const std::vector<int> &n0, const std::vector<int> &need0) {
  const int R = R_;
  auto ri = [&](int r, int i) { return rm_i_ + (size_t)r * kRmInts + i; };
  auto cand = [&](int r) { return cand_ + (size_t)r * cand_batch_ * kRmStride; };
  auto candv = [&](int r) { return cand_valid_ + (size_t)r * cand_batch_; };
  auto V = [&](int r) { return rm_V_ + (size_t)r * rm_cap_ * kRmStride; };
  std::vector<Cmd> grp;
  auto add = [&](Op op) -> Cmd & {
    grp.emplace_back();
    grp.back().op = op;
    return grp.back();
  };
  mrpop_status st;
  if (!act.empty()) {
    for (int r : act)
      add(Op::RmSample).rm_sample = RmSampleArgs{cand(r), cand_batch_, h_nj_[r], scene_->dev.q_lo + h_qoff_[r],
                                                 scene_->dev.q_hi + h_qoff_[r],
                                                 roadmap_key(P_.seed, (uint64_t)it * 1024 + g, (uint64_t)r), j0,
                                                 cand_codes_ + (size_t)r * cand_batch_,
                                                 speculative ? ri(r, 3) : nullptr};
    if ((st = group_(ex, grp)) != MRPOP_OK) return st;
    for (int r : act)  // consecutive validations: one launch over the arms
      if ((st = validate_(ex, arms_[r], cand(r), cand(r), cand_batch_, 1.0f, candv(r), cnt_ + (size_t)(2 + r) * 16,
                          cand_codes_ + (size_t)r * cand_batch_)) != MRPOP_OK)
        return st;
  }
  // acceptance (arms without samples this pass accept none), which also
  // zeroes the pair counters of every counted arm
  for (int r : counted) {
    const bool sampled = need[r] > 0 && std::find(act.begin(), act.end(), r) != act.end();
    add(Op::RmAccept).rm_accept =
        RmAcceptArgs{cand(r), candv(r), sampled ? cand_batch_ : 0, h_nj_[r], sampled ? need[r] : 0, V(r),
                     rm_nv_ + r, rm_cap_, ri(r, 0), uf_ + (size_t)r * rm_cap_, ri(r, 1),
                     speculative ? ri(r, 3) : nullptr};
  }
  if ((st = group_(ex, grp)) != MRPOP_OK) return st;
  for (int r : counted)
    add(Op::RmPairs).rm_pairs = RmPairsArgs{V(r), n0[r], n0[r] + need0[r], h_nj_[r], P_.delta, ri(r, 1), 0,
                                            nullptr, nullptr, nullptr, rm_nv_ + r, 0.f, nullptr};
  if ((st = group_(ex, grp)) != MRPOP_OK) return st;
  add(Op::Copy).copy = CopyArgs{pin_rm_, rm_i_, (int64_t)(sizeof(int32_t) * (size_t)R * kRmInts)};
  add(Op::Copy).copy = CopyArgs{pin_rm_ + (size_t)R * kRmInts, rm_nv_, (int64_t)(sizeof(int32_t) * (size_t)R)};
  return group_(ex, grp);
}

Task<mrpop_status> PlanJob::roadmap_(Exec &ex, int it) {
  const int R = R_;
  std::vector<char> conn(R, 0), grew(R, 0);
  std::vector<int> need(R, 0), need0(R, 0), n0(R, 0), np(R, 0), off(R, 0);
  auto ri = [&](int r, int i) { return rm_i_ + (size_t)r * kRmInts + i; };
  std::vector<Cmd> grp;
  auto add = [&](Op op) -> Cmd & {
    grp.emplace_back();
    grp.back().op = op;
    return grp.back();
  };
  // n free samples per arm and round, drawn in batches (the first free ones
  // in draw order); the arms of the round and those that still need samples
  auto begin_round = [&](const std::vector<int> &arms) {
    for (int r : arms) {
      n0[r] = rm_n_[r];
      need[r] = std::min(P_.n_roadmap, rm_cap_ - n0[r]);
      if (need[r] <= 0) st_.capacity_hit = 1;
      need0[r] = std::max(need[r], 0);
    }
  };
  auto needing = [&](const std::vector<int> &arms) {
    std::vector<int> a;
    for (int r : arms)
      if (need[r] > 0) a.push_back(r);
    return a;
  };
  auto take = [&](const std::vector<int> &arms) {  // a pass's accepted samples, from pinned memory
    for (int r : arms) {
      need[r] -= pin_rm_[(size_t)r * kRmInts];
      rm_n_[r] = pin_rm_[(size_t)R * kRmInts + r];
    }
  };
  if (P_.max_growth_rounds < 1) co_return MRPOP_OK;
  std::vector<int> todo;  // the arms that grow in this round
  for (int r = 0; r < R; ++r) todo.push_back(r);
  begin_round(todo);
  std::vector<int> act0 = needing(todo);  // the arms the round's first pass sampled
  TRY(rm_pass_(ex, it, 0, 0, act0, todo, false, need, n0, need0));
  SYNC();
  for (int g = 0;; ++g) {
    // the round's first pass (arms connected since took nothing), then more
    // passes while an arm lacks free samples (pair counts of the arms whose
    // vertices a pass changed, bounded by the vertex count on the device)
    take(act0);
    if (!act0.empty()) {
      for (int64_t j0 = cand_batch_;; j0 += cand_batch_) {
        const std::vector<int> act = needing(todo);
        if (act.empty()) break;
        TRY(rm_pass_(ex, it, g, j0, act, act, false, need, n0, need0));
        SYNC();
        take(act);
        if (j0 > (int64_t)cand_batch_ * 64) break;  // (nearly) no free space left
      }
    }
    // the pairs (the pair buffer shared in arm order), their validation, new
    // edges and the union of components; the union also writes each arm's
    // connectivity and validation counters to pinned memory
    int base = 0;
    for (int r : todo) {
      const int want = pin_rm_[(size_t)r * kRmInts + 1];
      np[r] = std::min(want, pair_cap_ - base);
      if (want > np[r]) st_.capacity_hit = 1;
      off[r] = base;
      base += np[r];
    }
    for (int r : todo)
      if (np[r] > 0)
        add(Op::RmPairs).rm_pairs =
            RmPairsArgs{rm_V_ + (size_t)r * rm_cap_ * kRmStride, n0[r], rm_n_[r], h_nj_[r], P_.delta, ri(r, 2), np[r],
                        pair_ids_ + 2 * (size_t)off[r], pair_qa_ + (size_t)off[r] * h_nj_[r],
                        pair_qb_ + (size_t)off[r] * h_nj_[r], nullptr, P_.resolution, pair_codes_ + off[r]};
    TRY(group_(ex, grp));
    for (int r : todo)
      if (np[r] > 0)
        TRY(validate_(ex, arms_[r], pair_qa_ + (size_t)off[r] * h_nj_[r], pair_qb_ + (size_t)off[r] * h_nj_[r],
                      np[r], P_.resolution, pair_valid_ + off[r], cnt_ + (size_t)(2 + r) * 16, pair_codes_ + off[r]));
    for (int r : todo) {
      if (np[r] > 0) grew[r] = 1;
      add(Op::RmUnion).rm_union =
          RmUnionArgs{pair_ids_ + 2 * (size_t)off[r], pair_valid_ + off[r], ri(r, 2), np[r], rm_n_[r],
                      uf_ + (size_t)r * rm_cap_, ri(r, 3),
                      np[r] > 0 ? rm_edges_ + (size_t)r * edge_cap_ * 2 : nullptr, rm_ne_ + r, edge_cap_,
                      pin_rm_ + (size_t)r * kRmInts + 3, np[r] > 0 ? cnt_ + (size_t)(2 + r) * 16 : nullptr,
                      pin_cnt_ + (size_t)r * 16};
    }
    TRY(group_(ex, grp));
    // the next round's first pass, queued behind the union
    const bool more = g + 1 < P_.max_growth_rounds && !out_of_time_();
    if (more) {
      begin_round(todo);
      act0 = needing(todo);
      TRY(rm_pass_(ex, it, g + 1, 0, act0, todo, true, need, n0, need0));
    }
    SYNC();
    bool all = true;
    for (int r : todo) {
      if (np[r] > 0) st_.roadmap_edge_states += (int64_t)pin_cnt_[(size_t)r * 16 + 1];
      conn[r] = (char)pin_rm_[(size_t)r * kRmInts + 3];
    }
    for (int r = 0; r < R; ++r) all = all && conn[r];
    if (all || !more) break;
    std::vector<int> next, next_act;
    for (int r : todo)
      if (!conn[r]) next.push_back(r);
    for (int r : act0)
      if (!conn[r]) next_act.push_back(r);
    todo.swap(next);
    act0.swap(next_act);
  }
  // adjacency (CSR) of the arms that gained edges
  for (int r = 0; r < R; ++r)
    if (grew[r])
      add(Op::RmBfs).rm_bfs = RmBfsArgs{rm_edges_ + (size_t)r * edge_cap_ * 2, rm_ne_ + r, edge_cap_, rm_n_[r],
                                        rm_rowptr_ + (size_t)r * (rm_cap_ + 1), rm_col_ + (size_t)r * col_cap_,
                                        col_cap_, deg_ + (size_t)r * rm_cap_, nullptr, nullptr};
  TRY(group_(ex, grp));
  st_.roadmap_connected = 1;
  for (int r = 0; r < R; ++r) st_.roadmap_connected = st_.roadmap_connected && conn[r];
  co_return MRPOP_OK;
}

// Sum of the Euclidean steps of a path [len][D], in double precision.
static double path_cost(const std::vector<float> &p, int D) {
  const size_t len = p.size() / D;
  double cost = 0.0;
  for (size_t k = 0; k + 1 < len; ++k) {
    double d2 = 0.0;
    for (int j = 0; j < D; ++j) {
      const double t = (double)p[(k + 1) * D + j] - (double)p[k * D + j];
      d2 += t * t;
    }
    cost += std::sqrt(d2);
  }
  return cost;
}

mrpop_status PlanJob::export_roadmaps(float *V, int32_t v_cap, int32_t *E, int32_t e_cap, int32_t *n_v,
                                      int32_t *n_e) {
  const int R = R_;
  std::vector<int32_t> ne((size_t)R, 0);
  hipError_t e = hipSetDevice(ctx_->device);
  if (e == hipSuccess && !P_.direct) e = hipMemcpy(ne.data(), rm_ne_, sizeof(int32_t) * R, hipMemcpyDeviceToHost);
  for (int r = 0; r < R && e == hipSuccess; ++r) {
    const int nv = P_.direct ? 0 : rm_n_[r];
    n_v[r] = nv;
    n_e[r] = ne[r];
    if (V && v_cap > 0 && nv > 0)
      e = hipMemcpy(V + (size_t)r * v_cap * kRmStride, rm_V_ + (size_t)r * rm_cap_ * kRmStride,
                    sizeof(float) * kRmStride * std::min(nv, v_cap), hipMemcpyDeviceToHost);
    if (e == hipSuccess && E && e_cap > 0 && ne[r] > 0)
      e = hipMemcpy(E + (size_t)r * e_cap * 2, rm_edges_ + (size_t)r * edge_cap_ * 2,
                    sizeof(int32_t) * 2 * std::min(std::min(ne[r], edge_cap_), e_cap), hipMemcpyDeviceToHost);
  }
  if (e != hipSuccess) return hip_fail_(e, "plan: roadmap export");
  return MRPOP_OK;
}

void PlanJob::set_incumbent(const std::vector<float> &path) {
  const float c = (float)path_cost(path, D_);
  if (c < c_best_) {
    c_best_ = c;
    best_path_ = path;
  }
}

mrpop_status PlanJob::run_blocking(Exec &ex) {
  Task<mrpop_status> t = run(ex);
  t.handle().resume();  // every synchronisation point is immediate on a blocking executor
  if (!t.done()) return fail_(MRPOP_E_DEVICE, "plan: suspended on a blocking executor");
  return t.result();
}

Task<mrpop_status> PlanJob::run(Exec &ex) {
  const int R = R_, D = D_, PC = PC_;
  t_start_ = now_s();
  synced_ = false;
  // uploads (independent copies into distinct buffers) and the endpoints
  std::vector<Cmd> grp;
  auto add_copy = [&](void *dst, const void *src, size_t bytes) {
    grp.emplace_back();
    grp.back().op = Op::Copy;
    grp.back().copy = CopyArgs{dst, src, (int64_t)bytes};
  };
  add_copy(qs_, upload_, sizeof(float) * D);
  add_copy(qg_, upload_ + D, sizeof(float) * D);
  add_copy(ea_, upload_, sizeof(float) * D);
  add_copy(ea_ + D, upload_ + D, sizeof(float) * D);
  add_copy(d_nj_, upload_i_, sizeof(int32_t) * R);
  add_copy(d_qoff_, upload_i_ + R, sizeof(int32_t) * R);
  add_copy(rm_nv_, upload_i_ + 2 * R, sizeof(int32_t) * R);
  add_copy(rm_ne_, upload_i_ + 3 * R, sizeof(int32_t) * R);
  for (int r = 0; r < R; ++r)
    add_copy(rm_V_ + (size_t)r * rm_cap_ * kRmStride, upload_ + 2 * D + (size_t)r * 2 * kRmStride,
             sizeof(float) * 2 * kRmStride);
  for (int r = 0; r < R; ++r) add_copy(uf_ + (size_t)r * rm_cap_, upload_i_ + 4 * R, 2 * sizeof(int32_t));
  grp.emplace_back();
  grp.back().op = Op::Fill;
  grp.back().fill = FillArgs{(uint32_t *)rm_rowptr_, 0u, (int64_t)R * (rm_cap_ + 1)};
  TRY(group_(ex, grp));
  TRY(validate_(ex, scene_, ea_, ea_, 2, 1.0f, valid_, cnt_));
  TRY(copy_(ex, pin_->valid2, valid_, 2));
  SYNC();
  if (!pin_->valid2[0]) co_return fail_(MRPOP_E_START_INVALID, "plan: start state collides");
  if (!pin_->valid2[1]) co_return fail_(MRPOP_E_GOAL_INVALID, "plan: goal state collides");

  int rnd = 0, it = 0;
  bool overflow_no_path = false, roadmap_full = false, trees_grown = false;
  std::vector<float> hpath;
  std::vector<int32_t> hvid;
  while (it < P_.max_iterations && rnd < P_.max_rounds && !out_of_time_()) {
    if (!P_.direct) {
      const mrpop_status rs = co_await roadmap_(ex, it);
      if (rs != MRPOP_OK) co_return rs;
      if (!st_.roadmap_connected) {
        // some arm's start and goal are still in different components, so
        // the tensor product holds no start-goal path: ROADMAP goes on
        // growing in the next iteration instead of a search that cannot end
        ++it;
        if (st_.capacity_hit) {
          roadmap_full = true;
          break;
        }
        continue;
      }
    }
    if (!P_.rewire || !trees_grown) {
      // fresh trees: 0 rooted at the start, 1 at the goal; a fresh search state
      SUBMIT(Op::TreeRoot, tree_root,
             TreeRootArgs{tq_[0], tg_[0], tvid_[0], tpar_[0], tn_[0], te_[0], tcap_, qs_, D, R, 0, ss_});
      SUBMIT(Op::TreeRoot, tree_root,
             TreeRootArgs{tq_[1], tg_[1], tvid_[1], tpar_[1], tn_[1], te_[1], tcap_, qg_, D, R, 1, nullptr});
      trees_grown = true;
    } else {  // ao-dRRT keeps its trees: the search goes on from them
      SUBMIT(Op::Fill, fill, FillArgs{(uint32_t *)&ss_->stop, 0u, 1});
    }
    const TreePair trees{{tq_[0], tq_[1]}, {tg_[0], tg_[1]}, {tvid_[0], tvid_[1]}, {tpar_[0], tpar_[1]},
                         {tn_[0], tn_[1]}, {te_[0], te_[1]}};
    const RewireArgs rw{P_.rewire, prop_z_, prop_cost_, prop_len_,
                        P_.rewire ? ea_ + (size_t)2 * PC * D : nullptr, P_.rewire ? eb_ + (size_t)2 * PC * D : nullptr,
                        P_.rewire ? codes_ext_ + 2 * PC : nullptr, P_.rewire ? valid_ + 2 * PC : nullptr, e_new_,
                        rw_key_};
    // AO-X: cost-bounded NEAREST and extension (c_rand) once there is a path;
    // ao-dRRT never bounds them
    const bool bounded = !P_.rewire;
    bool solved = false, full = false;
    while (!solved && rnd < P_.max_rounds && !out_of_time_()) {
      // kRoundsPerWait rounds queued back to back (at most the rounds left):
      // each round's back half picks the next round's tree on the device, and
      // the round that connects (or fills the tree) stops the rest
      const int K = std::min(kRoundsPerWait, P_.max_rounds - rnd);
      const float cb = c_best_;
      for (int k = 0; k < K; ++k) {
        // the tree fields below are replaced on the device by the search
        // state's choice (tree 0 stands in)
        const SampleNearArgs sn{SampleArgs{PC, D, cb, P_.seed, (uint64_t)(rnd + k), 0, scene_->dev.q_lo,
                                           scene_->dev.q_hi, qs_, qg_, tq_[0], tcap_, q_rand_, c_rand_},
                                NearestArgs{tq_[0], tg_[0], 1, D, 1, tcap_, q_rand_, D,
                                            bounded && cb < INFINITY ? c_rand_ : nullptr, PC, near_idx_}};
        // front half: sample, nearest, extension, then the connection search
        // and edge; one validation of both halves; back half: insertion and
        // selection
        SUBMIT(Op::RoundFront, round_front,
               RoundFrontArgs{sn,
                              ExtendArgs{PC, D, R, near_idx_, q_rand_, bounded && cb < INFINITY ? c_rand_ : nullptr, tq_[0],
                                         tvid_[0], tg_[0], tcap_, rm_V_, rm_rowptr_, rm_col_, rm_cap_, col_cap_,
                                         d_nj_, d_qoff_, q_new_, vid_new_, g_new_, alive_, ea_, eb_, P_.resolution,
                                         codes_ext_, P_.direct, P_.step},
                              cb, budget_,
                              NearestArgs{tq_[1], tg_[1], 1, D, 1, tcap_, q_new_, D, budget_, PC, conn_idx_},
                              ConnArgs{PC, D, conn_idx_, q_new_, tq_[1], tcap_, ca_, cb_, P_.resolution,
                                       codes_conn_},
                              trees, ss_, rw});
        TRY(validate_(ex, scene_, ea_, eb_, batch_rows_, P_.resolution, valid_, cnt_, codes_ext_));
        SUBMIT(Op::InsertSelect, insert_select,
               InsertSelectArgs{PC, D, R, alive_, valid_, cvalid_, q_new_, g_new_, vid_new_, near_idx_, conn_idx_,
                                trees, tcap_, ss_, ins_idx_, codes_conn_, cnt_, status_, &pin_->status[k],
                                seq_ + (uint32_t)k + 1u, rw});
        if (P_.rewire) SUBMIT(Op::Refresh, refresh, RefreshArgs{trees, status_, tcap_});
      }
      {
        const hipError_t e_ = co_await SyncPoint{ex, &pin_->status[K - 1].seq, seq_ + (uint32_t)K};
        if (e_ != hipSuccess) co_return hip_fail_(e_, "round status");
      }
      seq_ += (uint32_t)K;
      bool stopped = false, overflow = false;
      for (int k = 0; k < K && !stopped; ++k) {
        const RoundStatus rsx = pin_->status[k];
        if (rsx.skipped) break;
        st_.edge_states += rsx.states_ext + rsx.states_conn + rsx.states_rw;
        st_.speculative_edge_states += rsx.states_spec;
        st_.rewired += rsx.rewired;
        if (rsx.overflow) {
          st_.capacity_hit = 1;
          overflow = true;
        }
        ++rnd;
        stopped = rsx.found || rsx.overflow;
        if (!rsx.found) continue;
        const int a = rsx.a, b = 1 - rsx.a;
        SUBMIT(Op::Path, path,
               PathArgs{rsx.a_idx, rsx.b_idx, D, tcap_, path_max_, tpar_[a], tpar_[b], tq_[a], tq_[b], path_d_,
                        &pin_->ints[0], R, tvid_[a], tvid_[b], path_vid_d_});
        SYNC();
        const int len = pin_->ints[0];
        if (len > path_max_ || len < 2) {
          st_.capacity_hit = 1;
          continue;
        }
        const size_t need = (size_t)len * D, need_v = (size_t)len * R;
        const size_t bytes = sizeof(float) * need + sizeof(int32_t) * need_v;
        if (bytes > pin_path_cap_) {
          if (pin_path_) (void)hipHostFree(pin_path_);
          pin_path_ = nullptr;
          pin_path_cap_ = 0;
          const hipError_t e = hipHostMalloc((void **)&pin_path_, bytes);
          if (e != hipSuccess) co_return hip_fail_(e, "hipHostMalloc(path)");
          pin_path_cap_ = bytes;
        }
        int32_t *pin_vid = (int32_t *)(pin_path_ + need);
        TRY(copy_(ex, pin_path_, path_d_, sizeof(float) * need));
        TRY(copy_(ex, pin_vid, path_vid_d_, sizeof(int32_t) * need_v));
        SYNC();
        hpath.assign(pin_path_, pin_path_ + need);
        hvid.assign(pin_vid, pin_vid + need_v);
        if (a == 1) {  // tree 1 is rooted at the goal: orient start -> goal
          for (int x = 0, y = len - 1; x < y; ++x, --y) {
            std::swap_ranges(hpath.begin() + (size_t)x * D, hpath.begin() + (size_t)(x + 1) * D,
                             hpath.begin() + (size_t)y * D);
            std::swap_ranges(hvid.begin() + (size_t)x * R, hvid.begin() + (size_t)(x + 1) * R,
                             hvid.begin() + (size_t)y * R);
          }
        }
        const double cost = path_cost(hpath, D);
        if ((float)cost < c_best_) {  // strictly cheaper incumbents only
          c_best_ = (float)cost;
          best_path_ = hpath;
          history_.push_back(Incumbent{hpath, hvid, c_best_, elapsed_(), rnd - 1});
          if (st_.n_costs < 64) st_.costs[st_.n_costs++] = c_best_;
          ++st_.solutions;
          if (st_.first_round < 0) {
            st_.first_round = rnd - 1;
            st_.time_to_first_s = elapsed_();
          }
          solved = true;
        }
      }
      if (overflow && !solved) {
        overflow_no_path = best_path_.empty();
        full = true;
        break;
      }
      if (stopped && !solved) {  // a connection no cheaper in double precision: the search goes on
        grp.clear();
        grp.emplace_back();
        grp.back().op = Op::Fill;
        grp.back().fill = FillArgs{(uint32_t *)&ss_->stop, 0u, 1};
        TRY(group_(ex, grp));
      }
    }
    // a search ends unsolved only when its tree is full (rounds and time are
    // checked above): the next iteration grows the roadmaps and starts afresh
    ++it;
    if (P_.stop_at_first && solved) break;
    if (full && P_.rewire) break;  // its trees persist, and they are full
  }
  SYNC();  // a failure of queued work is reported here at the latest
  synced_ = true;
  st_.rounds = rnd;
  st_.iterations = it;
  for (int r = 0; r < R && !P_.direct; ++r) st_.roadmap_vertices += rm_n_[r];
  st_.total_time_s = elapsed_();
  if (best_path_.empty()) {
    if (roadmap_full) co_return fail_(MRPOP_E_CAPACITY, "plan: roadmap full before start and goal were connected");
    co_return overflow_no_path ? fail_(MRPOP_E_CAPACITY, "plan: search tree full before any solution")
                            : fail_(MRPOP_E_NO_SOLUTION, "plan: budget exhausted without a solution");
  }
  co_return MRPOP_OK;
}

#undef SUBMIT
#undef SYNC
#undef TRY

}  // namespace mrpop

#define HIP_TRY(expr, what)                               \
  do {                                                    \
    hipError_t e_ = (expr);                               \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, what); \
  } while (0)

extern "C" {

void mrpop_plan_params_default(mrpop_plan_params *p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->seed = 0;
  p->delta = 3.0f;
  p->n_roadmap = 32;
  p->candidates = 128;
  p->resolution = 0.05f;
  p->max_rounds = 1000;
  p->max_iterations = 8;
  p->max_growth_rounds = 16;
  p->direct = 0;
  p->step = 1.0f;
  p->time_budget_s = 0.0;
  p->max_tree_nodes = 65536;
  p->max_roadmap_nodes = 8192;
  p->stop_at_first = 0;
  p->rewire = 0;
  p->warm_cost = INFINITY;
}

mrpop_status mrpop_nearest(mrpop_ctx *ctx, const float *vertices, const float *costs, int64_t n_vertices, int32_t dim,
                           const float *queries, const float *budgets, int64_t n_queries, int32_t *out_idx,
                           void *stream) {
  if (!ctx) return fail(nullptr, MRPOP_E_INVALID_ARG, "nearest: ctx is NULL");
  if (n_vertices < 0 || n_queries < 0 || dim < 1 || dim > kMaxDof || n_vertices > 0x7fffffff ||
      n_queries > 0x7fffffff)
    return fail(ctx, MRPOP_E_INVALID_ARG, "nearest: sizes out of range");
  if (n_queries == 0) return MRPOP_OK;
  if (!queries || !out_idx || (n_vertices > 0 && !vertices))
    return fail(ctx, MRPOP_E_INVALID_ARG, "nearest: NULL buffer");
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  NearestArgs a{vertices, costs, n_vertices, dim, dim, 1, queries, dim, budgets, n_queries, out_idx};
  HIP_TRY(launch_nearest(a, (hipStream_t)stream), "nearest launch");
  return MRPOP_OK;
}

mrpop_status mrpop_extend(mrpop_ctx *ctx, const mrpop_scene *scene, const mrpop_extend_batch *b, void *stream) {
  if (!ctx) return fail(nullptr, MRPOP_E_INVALID_ARG, "extend: ctx is NULL");
  if (!scene || scene->ctx != ctx) return fail(ctx, MRPOP_E_INVALID_ARG, "extend: scene not from this ctx");
  if (!b) return fail(ctx, MRPOP_E_INVALID_ARG, "extend: batch is NULL");
  if (b->n < 0 || b->tree_cap < 1 || b->rm_cap < 1 || b->col_cap < 0)
    return fail(ctx, MRPOP_E_INVALID_ARG, "extend: sizes out of range");
  if (b->n == 0) return MRPOP_OK;
  if (!b->near_idx || !b->q_rand || !b->tree_q || !b->tree_g || !b->tree_vid || !b->rm_vertices || !b->rm_rowptr ||
      (b->col_cap > 0 && !b->rm_col) || !b->q_new || !b->vid_new || !b->g_new || !b->alive ||
      (!b->edge_a) != (!b->edge_b))
    return fail(ctx, MRPOP_E_INVALID_ARG, "extend: NULL buffer");
  if (b->n_states && !(b->resolution > 0.f && std::isfinite(b->resolution)))
    return fail(ctx, MRPOP_E_INVALID_ARG, "extend: resolution must be finite and > 0");
  const int R = scene->n_robots;
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  // the arms' joint counts and offsets for the kernel, in the context's scratch
  std::vector<int32_t> h((size_t)2 * R);
  for (int r = 0, off = 0; r < R; ++r) {
    h[r] = scene->nj[r];
    h[R + r] = off;
    off += scene->nj[r];
  }
  void *d = nullptr;
  mrpop_status st = scratch_slot(ctx, 4, sizeof(int32_t) * h.size(), &d);
  if (st != MRPOP_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipStreamSynchronize(s), "extend: wait for the stream");  // an earlier call may still read the slot
  HIP_TRY(hipMemcpy(d, h.data(), sizeof(int32_t) * h.size(), hipMemcpyHostToDevice), "extend: arm table");
  const int32_t *d_nj = (const int32_t *)d, *d_off = d_nj + R;
  ExtendArgs a{b->n,           scene->dof,      R,           b->near_idx,  b->q_rand,   b->c_rand,  b->tree_q,
               b->tree_vid,    b->tree_g,       b->tree_cap, b->rm_vertices, b->rm_rowptr, b->rm_col, b->rm_cap,
               b->col_cap,     d_nj,            d_off,       b->q_new,     b->vid_new,  b->g_new,   b->alive,
               b->edge_a,      b->edge_b,       b->resolution, b->n_states};
  HIP_TRY(launch_extend(a, s), "extend launch");
  return MRPOP_OK;
}

mrpop_status mrpop_sample(mrpop_ctx *ctx, const mrpop_scene *scene, const float *q_start, const float *q_goal,
                          const float *root, float c_best, uint64_t seed, uint64_t round, int64_t first, int64_t n,
                          float *out_q, float *out_c, void *stream) {
  if (!ctx) return fail(nullptr, MRPOP_E_INVALID_ARG, "sample: ctx is NULL");
  if (!scene || scene->ctx != ctx) return fail(ctx, MRPOP_E_INVALID_ARG, "sample: scene not from this ctx");
  if (n < 0 || n > 0x7fffffff || first < 0 || first > 0x7fffffff || std::isnan(c_best))
    return fail(ctx, MRPOP_E_INVALID_ARG, "sample: arguments out of range");
  if (n == 0) return MRPOP_OK;
  if (!q_start || !q_goal || !root || !out_q) return fail(ctx, MRPOP_E_INVALID_ARG, "sample: NULL buffer");
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  SampleArgs a{(int)n, scene->dof, c_best, seed, round, (int)first, scene->dev.q_lo, scene->dev.q_hi,
               q_start, q_goal, root, 1, out_q, out_c};
  HIP_TRY(launch_sample(a, (hipStream_t)stream), "sample launch");
  return MRPOP_OK;
}

}  // extern "C"

// Writes job's incumbents into hist, cheapest first, as many as fit, with
// their roadmap vertices and the roadmaps when asked for.
static mrpop_status write_history(PlanJob &job, mrpop_plan_history *hist) {
  const auto &h = job.history();
  hist->n_entries = (int32_t)h.size();
  hist->n_written = 0;
  const int D = job.dof(), R = job.n_robots();
  int64_t row = 0;
  if (hist->entry_cap > 0) hist->offsets[0] = 0;
  // discovery order has strictly decreasing costs: the ranking is its reverse
  for (int k = (int)h.size() - 1; k >= 0; --k) {
    const int n = hist->n_written;
    const int64_t len = (int64_t)(h[k].path.size() / D);
    if (n >= hist->entry_cap || row + len > hist->waypoint_cap) break;
    std::memcpy(hist->waypoints + row * D, h[k].path.data(), sizeof(float) * h[k].path.size());
    if (hist->vertex_ids) std::memcpy(hist->vertex_ids + row * R, h[k].vids.data(), sizeof(int32_t) * h[k].vids.size());
    row += len;
    hist->offsets[n + 1] = (int32_t)row;
    hist->costs[n] = h[k].cost;
    if (hist->found_s) hist->found_s[n] = h[k].found_s;
    if (hist->found_round) hist->found_round[n] = h[k].round;
    hist->n_written = n + 1;
  }
  if (hist->rm_vertices || hist->rm_edges)
    return job.export_roadmaps(hist->rm_vertices, hist->rm_vertex_cap, hist->rm_edges, hist->rm_edge_cap,
                               hist->rm_n_vertices, hist->rm_n_edges);
  for (int r = 0; r < R; ++r) hist->rm_n_vertices[r] = hist->rm_n_edges[r] = 0;
  return MRPOP_OK;
}

static mrpop_status plan_impl(mrpop_ctx *ctx, const mrpop_scene *scene, const float *q_start, const float *q_goal,
                              const mrpop_plan_params *params, float *path_out, int32_t path_cap, int32_t *path_len,
                              float *cost_out, mrpop_plan_stats *stats_opt, mrpop_plan_history *hist,
                              const std::vector<float> *incumbent = nullptr) {
  if (!ctx) return fail(nullptr, MRPOP_E_INVALID_ARG, "plan: ctx is NULL");
  if (!scene || scene->ctx != ctx) return fail(ctx, MRPOP_E_INVALID_ARG, "plan: scene not from this ctx");
  if (!q_start || !q_goal || !params || !path_len || !cost_out || (path_cap > 0 && !path_out))
    return fail(ctx, MRPOP_E_INVALID_ARG, "plan: NULL argument");
  if (hist) {
    hist->n_entries = hist->n_written = 0;
    if (hist->entry_cap < 0 || hist->waypoint_cap < 0 ||
        (hist->entry_cap > 0 && (!hist->offsets || !hist->costs)) || (hist->waypoint_cap > 0 && !hist->waypoints) ||
        (hist->rm_vertices && hist->rm_vertex_cap < 1) || (hist->rm_edges && hist->rm_edge_cap < 1))
      return fail(ctx, MRPOP_E_INVALID_ARG, "plan: bad history buffers");
  }
  *path_len = 0;
  *cost_out = INFINITY;
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  PlanJob job;
  mrpop_status st = job.prepare(ctx, scene, q_start, q_goal, *params);
  if (st == MRPOP_OK) {
    if (incumbent) job.set_incumbent(*incumbent);
    PlainExec ex(ctx, nullptr);
    st = job.run_blocking(ex);
    if (hist) {
      const mrpop_status hs = write_history(job, hist);
      if (st == MRPOP_OK && hs != MRPOP_OK) st = hs;
    }
  }
  if (stats_opt) *stats_opt = job.stats();
  if (st != MRPOP_OK) return fail(ctx, st, job.error());
  const int len = (int)(job.path().size() / job.dof());
  *path_len = len;
  *cost_out = job.cost();
  if (len > path_cap) return fail(ctx, MRPOP_E_BUFFER, "plan: path buffer too small");
  std::memcpy(path_out, job.path().data(), sizeof(float) * job.path().size());
  return MRPOP_OK;
}

extern "C" {

mrpop_status mrpop_plan(mrpop_ctx *ctx, const mrpop_scene *scene, const float *q_start, const float *q_goal,
                        const mrpop_plan_params *params, float *path_out, int32_t path_cap, int32_t *path_len,
                        float *cost_out, mrpop_plan_stats *stats_opt) {
  return plan_impl(ctx, scene, q_start, q_goal, params, path_out, path_cap, path_len, cost_out, stats_opt, nullptr);
}

mrpop_status mrpop_replan(mrpop_ctx *ctx, const mrpop_scene *scene, const float *q_start, const float *q_goal,
                          const mrpop_plan_params *params, const float *prev_path, int32_t prev_len,
                          float *path_out, int32_t path_cap, int32_t *path_len, float *cost_out,
                          mrpop_plan_stats *stats_opt, int32_t *prev_valid_out) {
  if (prev_valid_out) *prev_valid_out = 0;
  if (!ctx) return fail(nullptr, MRPOP_E_INVALID_ARG, "replan: ctx is NULL");
  if (!scene || scene->ctx != ctx) return fail(ctx, MRPOP_E_INVALID_ARG, "replan: scene not from this ctx");
  if (!q_start || !q_goal || !params || prev_len < 0 || (prev_len > 0 && !prev_path))
    return fail(ctx, MRPOP_E_INVALID_ARG, "replan: bad argument");
  const int D = scene->dof;
  std::vector<float> warm;
  if (prev_len >= 2 && std::memcmp(prev_path, q_start, sizeof(float) * D) == 0 &&
      std::memcmp(prev_path + (size_t)(prev_len - 1) * D, q_goal, sizeof(float) * D) == 0 &&
      params->resolution > 0.f && std::isfinite(params->resolution)) {
    // the previous path's edges in the current environment
    const int64_t n = prev_len - 1;
    const size_t fb = sizeof(float) * (size_t)n * D;
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    void *buf = nullptr;
    HIP_TRY(hipMalloc(&buf, 2 * fb + (size_t)n), "hipMalloc(replan)");
    float *qa = (float *)buf, *qb = (float *)((unsigned char *)buf + fb);
    uint8_t *ok = (uint8_t *)buf + 2 * fb;
    std::vector<uint8_t> h_ok((size_t)n);
    hipError_t e = hipMemcpy(qa, prev_path, fb, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(qb, prev_path + D, fb, hipMemcpyHostToDevice);
    mrpop_status vs = MRPOP_E_DEVICE;
    if (e == hipSuccess) vs = mrpop_validate_edges(ctx, scene, qa, qb, n, params->resolution, nullptr, ok, nullptr, nullptr);
    if (vs == MRPOP_OK) e = hipMemcpy(h_ok.data(), ok, (size_t)n, hipMemcpyDeviceToHost);
    (void)hipFree(buf);
    if (vs != MRPOP_OK) return vs;
    if (e != hipSuccess) return hip_fail(ctx, e, "replan: validation copy");
    bool all = true;
    for (uint8_t v : h_ok) all = all && v == 1;
    if (all) warm.assign(prev_path, prev_path + (size_t)prev_len * D);
  }
  if (prev_valid_out) *prev_valid_out = warm.empty() ? 0 : 1;
  return plan_impl(ctx, scene, q_start, q_goal, params, path_out, path_cap, path_len, cost_out, stats_opt, nullptr,
                   warm.empty() ? nullptr : &warm);
}

mrpop_status mrpop_plan_with_history(mrpop_ctx *ctx, const mrpop_scene *scene, const float *q_start,
                                     const float *q_goal, const mrpop_plan_params *params, float *path_out,
                                     int32_t path_cap, int32_t *path_len, float *cost_out,
                                     mrpop_plan_stats *stats_opt, mrpop_plan_history *hist) {
  if (!hist) return fail(ctx, MRPOP_E_INVALID_ARG, "plan_with_history: hist is NULL");
  return plan_impl(ctx, scene, q_start, q_goal, params, path_out, path_cap, path_len, cost_out, stats_opt, hist);
}

}  // extern "C"
