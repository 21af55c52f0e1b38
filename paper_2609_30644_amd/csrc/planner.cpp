// MR. POP planner driver (Alg. 1) and the search-primitive entry points.
//
// The driver keeps every roadmap and both search trees on the device and
// runs the search in bulk-synchronous rounds of P candidates:
//   sample -> NEAREST in the extended tree -> dRRT oracle -> validate the
//   extensions -> insert in candidate order -> NEAREST in the other tree ->
//   validate the connections -> pick the cheapest connection.
// One small status record per round comes back to the host (pinned memory),
// which decides whether the search ended, swaps the trees when the extended
// one has grown larger, and extracts a path on success.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "planner.h"

using namespace mrpop;

namespace {

struct Arena {
  std::vector<std::pair<void **, size_t>> items;
  template <class T>
  void add(T **p, size_t n) {
    items.push_back({(void **)p, std::max<size_t>(n, 1) * sizeof(T)});
  }
  void *base = nullptr;
  hipError_t alloc() {
    size_t total = 0;
    for (auto &it : items) total += (it.second + 255) & ~size_t(255);
    hipError_t e = hipMalloc(&base, total);
    if (e != hipSuccess) {
      base = nullptr;
      return e;
    }
    size_t off = 0;
    for (auto &it : items) {
      *it.first = (unsigned char *)base + off;
      off += (it.second + 255) & ~size_t(255);
    }
    return hipSuccess;
  }
  ~Arena() {
    if (base) (void)hipFree(base);
  }
};

struct PinnedStatus {
  RoundStatus *h = nullptr;
  int32_t *ints = nullptr;
  ~PinnedStatus() {
    if (h) (void)hipHostFree(h);
    if (ints) (void)hipHostFree(ints);
  }
};

struct SceneHolder {
  mrpop_scene *s = nullptr;
  ~SceneHolder() {
    if (s) mrpop_scene_destroy(s);
  }
};

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

}  // namespace

#define HIP_TRY(expr, what)                      \
  do {                                           \
    hipError_t e_ = (expr);                      \
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
  p->time_budget_s = 0.0;
  p->max_tree_nodes = 65536;
  p->max_roadmap_nodes = 8192;
  p->stop_at_first = 0;
  p->warm_cost = INFINITY;
}

mrpop_status mrpop_nearest(mrpop_ctx *ctx, const float *vertices, const float *costs, int64_t n_vertices, int32_t dim,
                           const float *queries, const float *budgets, int64_t n_queries, int32_t *out_idx,
                           void *stream) {
  if (!ctx) return fail(nullptr, MRPOP_E_INVALID_ARG, "nearest: ctx is NULL");
  if (n_vertices < 0 || n_queries < 0 || dim < 1 || dim > kMaxDof || n_vertices > 0x7fffffff)
    return fail(ctx, MRPOP_E_INVALID_ARG, "nearest: sizes out of range");
  if (n_queries == 0) return MRPOP_OK;
  if (!queries || !out_idx || (n_vertices > 0 && !vertices))
    return fail(ctx, MRPOP_E_INVALID_ARG, "nearest: NULL buffer");
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  NearestArgs a{vertices, costs, n_vertices, dim, dim, 1, queries, dim, budgets, n_queries, out_idx};
  HIP_TRY(launch_nearest(a, (hipStream_t)stream), "nearest launch");
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

mrpop_status mrpop_plan(mrpop_ctx *ctx, const mrpop_scene *scene, const float *q_start, const float *q_goal,
                        const mrpop_plan_params *params, float *path_out, int32_t path_cap, int32_t *path_len,
                        float *cost_out, mrpop_plan_stats *stats_opt) {
  if (!ctx) return fail(nullptr, MRPOP_E_INVALID_ARG, "plan: ctx is NULL");
  if (!scene || scene->ctx != ctx) return fail(ctx, MRPOP_E_INVALID_ARG, "plan: scene not from this ctx");
  if (!q_start || !q_goal || !params || !path_len || !cost_out || (path_cap > 0 && !path_out))
    return fail(ctx, MRPOP_E_INVALID_ARG, "plan: NULL argument");
  const mrpop_plan_params &P = *params;
  if (P.candidates < 1 || P.candidates > 4096 || !(P.resolution > 0.f) || !std::isfinite(P.resolution) ||
      P.max_rounds < 1 || P.max_iterations < 1 || P.max_growth_rounds < 1 || P.n_roadmap < 1 ||
      P.max_tree_nodes < 2 || P.max_roadmap_nodes < 4 || !(P.delta > 0.f) || P.time_budget_s < 0 ||
      std::isnan(P.warm_cost))
    return fail(ctx, MRPOP_E_INVALID_ARG, "plan: parameter out of range");
  const int R = scene->n_robots, D = scene->dof, PC = P.candidates;
  for (int j = 0; j < D; ++j)
    if (!std::isfinite(q_start[j]) || !std::isfinite(q_goal[j]))
      return fail(ctx, MRPOP_E_NONFINITE, "plan: non-finite start or goal");
  *path_len = 0;
  *cost_out = INFINITY;
  mrpop_plan_stats st;
  std::memset(&st, 0, sizeof(st));
  st.time_to_first_s = -1.0;
  st.first_round = -1;
  const double t_start = now_s();
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  hipStream_t s = nullptr;

  // ---- device buffers ----------------------------------------------------
  const int rm_cap = P.max_roadmap_nodes, edge_cap = rm_cap * 32, col_cap = 2 * edge_cap;
  const int cand_batch = 4 * P.n_roadmap;
  const int pair_cap = P.n_roadmap * rm_cap;
  const int tcap = P.max_tree_nodes;
  const int path_max = 16384;
  int max_nj = 0;
  for (int r = 0; r < R; ++r) max_nj = std::max(max_nj, scene->nj[r]);
  Arena ar;
  float *qs, *qg, *rm_V, *cand, *pair_qa, *pair_qb, *tq[2], *tg[2], *q_rand, *c_rand, *q_new, *g_new, *ea, *eb,
      *budget, *ca, *cb, *path;
  int32_t *rm_rowptr, *rm_col, *rm_edges, *rm_nv, *rm_ne, *pair_ids, *pair_count, *taken, *connected, *deg, *level,
      *tvid[2], *tpar[2], *tn[2], *near_idx, *vid_new, *ins_idx, *conn_idx, *path_len_d, *d_nj, *d_qoff;
  uint8_t *cand_valid, *pair_valid, *alive, *valid, *cvalid;
  RoundStatus *status;
  ar.add(&qs, D);
  ar.add(&qg, D);
  ar.add(&rm_V, (size_t)R * rm_cap * kRmStride);
  ar.add(&rm_rowptr, (size_t)R * (rm_cap + 1));
  ar.add(&rm_col, (size_t)R * col_cap);
  ar.add(&rm_edges, (size_t)R * edge_cap * 2);
  ar.add(&rm_nv, R);
  ar.add(&rm_ne, R);
  ar.add(&cand, (size_t)cand_batch * kRmStride);
  ar.add(&cand_valid, cand_batch);
  ar.add(&pair_ids, (size_t)pair_cap * 2);
  ar.add(&pair_qa, (size_t)pair_cap * max_nj);
  ar.add(&pair_qb, (size_t)pair_cap * max_nj);
  ar.add(&pair_valid, pair_cap);
  ar.add(&pair_count, 1);
  ar.add(&taken, 1);
  ar.add(&connected, 1);
  ar.add(&deg, rm_cap);
  ar.add(&level, rm_cap);
  for (int t = 0; t < 2; ++t) {
    ar.add(&tq[t], (size_t)D * tcap);
    ar.add(&tg[t], tcap);
    ar.add(&tvid[t], (size_t)R * tcap);
    ar.add(&tpar[t], tcap);
    ar.add(&tn[t], 1);
  }
  ar.add(&q_rand, (size_t)PC * D);
  ar.add(&c_rand, PC);
  ar.add(&near_idx, PC);
  ar.add(&q_new, (size_t)PC * D);
  ar.add(&g_new, PC);
  ar.add(&vid_new, (size_t)R * PC);
  ar.add(&alive, PC);
  ar.add(&ea, (size_t)PC * D);
  ar.add(&eb, (size_t)PC * D);
  ar.add(&valid, PC);
  ar.add(&ins_idx, PC);
  ar.add(&budget, PC);
  ar.add(&conn_idx, PC);
  ar.add(&ca, (size_t)PC * D);
  ar.add(&cb, (size_t)PC * D);
  ar.add(&cvalid, PC);
  ar.add(&status, 1);
  ar.add(&path, (size_t)path_max * D);
  ar.add(&path_len_d, 1);
  ar.add(&d_nj, R);
  ar.add(&d_qoff, R);
  HIP_TRY(ar.alloc(), "hipMalloc(plan)");
  PinnedStatus pin;
  HIP_TRY(hipHostMalloc((void **)&pin.h, sizeof(RoundStatus)), "hipHostMalloc");
  HIP_TRY(hipHostMalloc((void **)&pin.ints, 4 * sizeof(int32_t)), "hipHostMalloc");

  std::vector<int32_t> h_qoff(R), h_nj(R);
  for (int r = 0, o = 0; r < R; ++r) {
    h_qoff[r] = o;
    h_nj[r] = scene->nj[r];
    o += scene->nj[r];
  }
  HIP_TRY(hipMemcpy(qs, q_start, sizeof(float) * D, hipMemcpyHostToDevice), "copy");
  HIP_TRY(hipMemcpy(qg, q_goal, sizeof(float) * D, hipMemcpyHostToDevice), "copy");
  HIP_TRY(hipMemcpy(d_nj, h_nj.data(), sizeof(int32_t) * R, hipMemcpyHostToDevice), "copy");
  HIP_TRY(hipMemcpy(d_qoff, h_qoff.data(), sizeof(int32_t) * R, hipMemcpyHostToDevice), "copy");

  // ---- validation helper (separate scratch per use) -----------------------
  auto validate = [&](const mrpop_scene *sc, const float *a, const float *b, int64_t n, float res, uint8_t *out,
                      int slot, uint64_t **counters) -> mrpop_status {
    void *base = nullptr;
    mrpop_status st2 = scratch(ctx, slot, validate_scratch_bytes(std::max<int64_t>(n, 1)), &base);
    if (st2 != MRPOP_OK) return st2;
    ValidateScratch ws = validate_scratch_layout(base, std::max<int64_t>(n, 1));
    if (counters) *counters = ws.counters;
    if (n == 0) return MRPOP_OK;
    hipError_t e = launch_validate(sc->dev, a, b, n, res, nullptr, out, ws, s, profile_slot(ctx),
                                   ctx->profiling ? ctx->prof_totals : nullptr, &ctx->last_grid, &ctx->last_block);
    return e == hipSuccess ? MRPOP_OK : hip_fail(ctx, e, "validate launch");
  };

  // ---- endpoints -----------------------------------------------------------
  {
    HIP_TRY(hipMemcpy(ea, q_start, sizeof(float) * D, hipMemcpyHostToDevice), "copy");
    HIP_TRY(hipMemcpy(ea + D, q_goal, sizeof(float) * D, hipMemcpyHostToDevice), "copy");
    mrpop_status v = validate(scene, ea, ea, 2, 1.0f, valid, 1, nullptr);
    if (v != MRPOP_OK) return v;
    uint8_t ok[2];
    HIP_TRY(hipMemcpy(ok, valid, 2, hipMemcpyDeviceToHost), "copy");
    if (!ok[0]) return fail(ctx, MRPOP_E_START_INVALID, "plan: start state collides");
    if (!ok[1]) return fail(ctx, MRPOP_E_GOAL_INVALID, "plan: goal state collides");
  }

  // ---- roadmaps: vertex 0 = the arm's start, vertex 1 = its goal -----------
  std::vector<SceneHolder> arms(R);
  for (int r = 0; r < R; ++r) {
    mrpop_status a = arm_scene(ctx, scene, r, &arms[r].s);
    if (a != MRPOP_OK) return a;
  }
  std::vector<int32_t> rm_n(R, 2);
  {
    std::vector<float> init((size_t)R * 2 * kRmStride, 0.f);
    for (int r = 0; r < R; ++r)
      for (int j = 0; j < h_nj[r]; ++j) {
        init[((size_t)r * 2 + 0) * kRmStride + j] = q_start[h_qoff[r] + j];
        init[((size_t)r * 2 + 1) * kRmStride + j] = q_goal[h_qoff[r] + j];
      }
    for (int r = 0; r < R; ++r)
      HIP_TRY(hipMemcpy(rm_V + (size_t)r * rm_cap * kRmStride, &init[(size_t)r * 2 * kRmStride],
                        sizeof(float) * 2 * kRmStride, hipMemcpyHostToDevice),
              "copy");
    std::vector<int32_t> two(R, 2), zero(R, 0);
    HIP_TRY(hipMemcpy(rm_nv, two.data(), sizeof(int32_t) * R, hipMemcpyHostToDevice), "copy");
    HIP_TRY(hipMemcpy(rm_ne, zero.data(), sizeof(int32_t) * R, hipMemcpyHostToDevice), "copy");
    HIP_TRY(hipMemset(rm_rowptr, 0, sizeof(int32_t) * (size_t)R * (rm_cap + 1)), "memset");
  }

  auto elapsed = [&]() { return now_s() - t_start; };
  auto out_of_time = [&]() { return P.time_budget_s > 0 && elapsed() >= P.time_budget_s; };

  // ROADMAP (Alg. 2) for outer iteration `it`
  auto roadmap = [&](int it) -> mrpop_status {
    std::vector<char> conn(R, 0);
    for (int g = 0; g < P.max_growth_rounds; ++g) {
      bool all = true;
      for (int r = 0; r < R; ++r) {
        if (conn[r]) continue;
        const int nj = h_nj[r];
        float *V = rm_V + (size_t)r * rm_cap * kRmStride;
        const int n0 = rm_n[r];
        int need = std::min(P.n_roadmap, rm_cap - n0);
        if (need <= 0) st.capacity_hit = 1;
        for (int64_t j0 = 0; need > 0; j0 += cand_batch) {
          HIP_TRY(launch_rm_sample(cand, cand_batch, nj, scene->dev.q_lo + h_qoff[r], scene->dev.q_hi + h_qoff[r],
                                   P.seed, (uint64_t)it * 1024 + g, (uint64_t)r, j0, s),
                  "rm_sample");
          mrpop_status v = validate(arms[r].s, cand, cand, cand_batch, 1.0f, cand_valid, 3, nullptr);
          if (v != MRPOP_OK) return v;
          HIP_TRY(launch_rm_accept(cand, cand_valid, cand_batch, nj, need, V, rm_nv + r, rm_cap, taken, s),
                  "rm_accept");
          HIP_TRY(hipMemcpyAsync(pin.ints, taken, sizeof(int32_t), hipMemcpyDeviceToHost, s), "copy");
          HIP_TRY(hipStreamSynchronize(s), "sync");
          need -= pin.ints[0];
          if (j0 > (int64_t)cand_batch * 64) break;  // the arm's free space is (nearly) empty
        }
        HIP_TRY(hipMemcpyAsync(pin.ints, rm_nv + r, sizeof(int32_t), hipMemcpyDeviceToHost, s), "copy");
        HIP_TRY(hipStreamSynchronize(s), "sync");
        rm_n[r] = pin.ints[0];
        // candidate edges between the new vertices and all earlier ones
        HIP_TRY(hipMemsetAsync(pair_count, 0, sizeof(int32_t), s), "memset");
        HIP_TRY(launch_rm_pairs(V, n0, rm_n[r], nj, P.delta, pair_count, pair_cap, pair_ids, pair_qa, pair_qb, s),
                "rm_pairs");
        HIP_TRY(hipMemcpyAsync(pin.ints, pair_count, sizeof(int32_t), hipMemcpyDeviceToHost, s), "copy");
        HIP_TRY(hipStreamSynchronize(s), "sync");
        const int np = std::min(pin.ints[0], pair_cap);
        if (pin.ints[0] > pair_cap) st.capacity_hit = 1;
        uint64_t *cnt = nullptr;
        mrpop_status v = validate(arms[r].s, pair_qa, pair_qb, np, P.resolution, pair_valid, 4, &cnt);
        if (v != MRPOP_OK) return v;
        if (np > 0) {
          HIP_TRY(launch_rm_add_edges(pair_ids, pair_valid, pair_count, np, rm_edges + (size_t)r * edge_cap * 2,
                                      rm_ne + r, edge_cap, s),
                  "rm_add_edges");
          uint64_t c2[2];
          HIP_TRY(hipMemcpyAsync(c2, cnt, sizeof(c2), hipMemcpyDeviceToHost, s), "copy");
          HIP_TRY(hipStreamSynchronize(s), "sync");
          st.roadmap_edge_states += (int64_t)c2[1];
        }
        HIP_TRY(launch_rm_csr_bfs(rm_edges + (size_t)r * edge_cap * 2, rm_ne + r, edge_cap, rm_n[r],
                                  rm_rowptr + (size_t)r * (rm_cap + 1), rm_col + (size_t)r * col_cap, col_cap, deg,
                                  level, connected, s),
                "rm_csr_bfs");
        HIP_TRY(hipMemcpyAsync(pin.ints, connected, sizeof(int32_t), hipMemcpyDeviceToHost, s), "copy");
        HIP_TRY(hipStreamSynchronize(s), "sync");
        conn[r] = (char)pin.ints[0];
        all = all && conn[r];
      }
      if (all) break;
      if (out_of_time()) break;
    }
    st.roadmap_connected = 1;
    for (int r = 0; r < R; ++r) st.roadmap_connected = st.roadmap_connected && conn[r];
    return MRPOP_OK;
  };

  float c_best = P.warm_cost;
  std::vector<float> best_path;
  int rnd = 0, it = 0;
  bool overflow_no_path = false;
  std::vector<float> hpath;
  while (it < P.max_iterations && rnd < P.max_rounds && !out_of_time()) {
    mrpop_status rs = roadmap(it);
    if (rs != MRPOP_OK) return rs;
    // fresh trees: 0 rooted at the start, 1 at the goal
    HIP_TRY(launch_tree_root(tq[0], tvid[0], tg[0], tpar[0], tn[0], tcap, qs, D, R, 0, s), "tree_root");
    HIP_TRY(launch_tree_root(tq[1], tvid[1], tg[1], tpar[1], tn[1], tcap, qg, D, R, 1, s), "tree_root");
    int n_t[2] = {1, 1};
    int a = 0;  // index of the tree being extended
    bool solved = false;
    while (!solved && rnd < P.max_rounds && !out_of_time()) {
      if (n_t[a] > n_t[1 - a]) a = 1 - a;
      const int b = 1 - a;
      SampleArgs sa{PC, D, c_best, P.seed, (uint64_t)rnd, 0, scene->dev.q_lo, scene->dev.q_hi, qs, qg, tq[a], tcap,
                    q_rand, c_rand};
      HIP_TRY(launch_sample(sa, s), "sample");
      NearestArgs na{tq[a], tg[a], n_t[a], D, 1, tcap, q_rand, D, c_best < INFINITY ? c_rand : nullptr, PC, near_idx};
      HIP_TRY(launch_nearest(na, s), "nearest");
      ExtendArgs xa{PC, D, R, near_idx, q_rand, c_best < INFINITY ? c_rand : nullptr, tq[a], tvid[a], tg[a], tcap,
                    rm_V, rm_rowptr, rm_col, rm_cap, col_cap, d_nj, d_qoff, q_new, vid_new, g_new, alive, ea, eb};
      HIP_TRY(launch_extend(xa, s), "extend");
      uint64_t *cnt_ext = nullptr, *cnt_conn = nullptr;
      mrpop_status v = validate(scene, ea, eb, PC, P.resolution, valid, 1, &cnt_ext);
      if (v != MRPOP_OK) return v;
      InsertArgs ia{PC, D, R, alive, valid, q_new, g_new, vid_new, near_idx, tq[a], tg[a], tvid[a], tpar[a], tn[a],
                    tcap, c_best, ins_idx, budget, status};
      HIP_TRY(launch_insert(ia, s), "insert");
      NearestArgs nb{tq[b], tg[b], n_t[b], D, 1, tcap, q_new, D, budget, PC, conn_idx};
      HIP_TRY(launch_nearest(nb, s), "nearest");
      ConnArgs cna{PC, D, conn_idx, q_new, tq[b], tcap, ca, cb};
      HIP_TRY(launch_conn_edges(cna, s), "conn_edges");
      v = validate(scene, ca, cb, PC, P.resolution, cvalid, 2, &cnt_conn);
      if (v != MRPOP_OK) return v;
      SelectArgs sl{PC, D, ins_idx, conn_idx, cvalid, q_new, g_new, tq[b], tg[b], tcap, cnt_ext, cnt_conn, status};
      HIP_TRY(launch_select(sl, s), "select");
      HIP_TRY(hipMemcpyAsync(pin.h, status, sizeof(RoundStatus), hipMemcpyDeviceToHost, s), "copy");
      HIP_TRY(hipStreamSynchronize(s), "sync");
      const RoundStatus rsx = *pin.h;
      st.edge_states += rsx.states_ext + rsx.states_conn;
      n_t[a] += rsx.inserted;
      if (rsx.overflow) st.capacity_hit = 1;
      ++rnd;
      if (rsx.found) {
        PathArgs pa{rsx.a_idx, rsx.b_idx, D, tcap, path_max, tpar[a], tpar[b], tq[a], tq[b], path, path_len_d};
        HIP_TRY(launch_path(pa, s), "path");
        HIP_TRY(hipMemcpyAsync(pin.ints, path_len_d, sizeof(int32_t), hipMemcpyDeviceToHost, s), "copy");
        HIP_TRY(hipStreamSynchronize(s), "sync");
        const int len = pin.ints[0];
        if (len > path_max || len < 2) {
          st.capacity_hit = 1;
        } else {
          hpath.resize((size_t)len * D);
          HIP_TRY(hipMemcpy(hpath.data(), path, sizeof(float) * len * D, hipMemcpyDeviceToHost), "copy");
          if (a == 1) {  // tree 1 is rooted at the goal: orient start -> goal
            for (int x = 0, y = len - 1; x < y; ++x, --y)
              std::swap_ranges(hpath.begin() + (size_t)x * D, hpath.begin() + (size_t)(x + 1) * D,
                               hpath.begin() + (size_t)y * D);
          }
          double cost = 0.0;
          for (int k = 0; k + 1 < len; ++k) {
            double d2 = 0.0;
            for (int j = 0; j < D; ++j) {
              const double t = (double)hpath[(size_t)(k + 1) * D + j] - (double)hpath[(size_t)k * D + j];
              d2 += t * t;
            }
            cost += std::sqrt(d2);
          }
          if ((float)cost < c_best) {  // strictly cheaper incumbents only
            c_best = (float)cost;
            best_path = hpath;
            if (st.n_costs < 64) st.costs[st.n_costs++] = c_best;
            ++st.solutions;
            if (st.first_round < 0) {
              st.first_round = rnd - 1;
              st.time_to_first_s = elapsed();
            }
            solved = true;
          }
        }
      }
      if (rsx.overflow && !solved) {
        overflow_no_path = best_path.empty();
        break;
      }
    }
    ++it;
    if (!solved) break;
    if (P.stop_at_first && !best_path.empty()) break;
  }
  st.rounds = rnd;
  st.iterations = it;
  for (int r = 0; r < R; ++r) st.roadmap_vertices += rm_n[r];
  st.total_time_s = elapsed();
  if (stats_opt) *stats_opt = st;
  if (best_path.empty())
    return overflow_no_path ? fail(ctx, MRPOP_E_CAPACITY, "plan: search tree full before any solution")
                            : fail(ctx, MRPOP_E_NO_SOLUTION, "plan: budget exhausted without a solution");
  const int len = (int)(best_path.size() / D);
  *path_len = len;
  *cost_out = c_best;
  if (len > path_cap) return fail(ctx, MRPOP_E_BUFFER, "plan: path buffer too small");
  std::memcpy(path_out, best_path.data(), sizeof(float) * best_path.size());
  return MRPOP_OK;
}

}  // extern "C"
