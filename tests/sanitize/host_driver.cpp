// Drives the library's host runtime through every C entry point on a small
// two-arm scene, for a build whose host code carries AddressSanitizer and
// UndefinedBehaviorSanitizer (the device code is built as usual).  Any
// finding aborts the run; the program prints "host driver ok" at the end.
// Checks here are coarse (statuses, a few equalities): the numerics are the
// parity tests' job.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "mrpop.h"

#define CHECK(cond)                                                               \
  do {                                                                            \
    if (!(cond)) {                                                                \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond);     \
      std::exit(1);                                                               \
    }                                                                             \
  } while (0)
#define HIPCHECK(expr) CHECK((expr) == hipSuccess)

namespace {

// a small fixed generator (xorshift64*), so that runs are reproducible
struct Rng {
  uint64_t s;
  double u() {
    s ^= s >> 12;
    s ^= s << 25;
    s ^= s >> 27;
    return (double)((s * 2685821657736338717ull) >> 11) * (1.0 / 9007199254740992.0);
  }
};

// A Panda-like arm: modified DH rows (a_{j-1}, d_j, alpha_{j-1}, theta_off),
// the manufacturer's limits, and 2 spheres per link.
struct Arm {
  float dh[7 * 4] = {0.f,     0.333f, 0.f,        0.f, 0.f,     0.f,    -1.5707963f, 0.f,
                     0.f,     0.316f, 1.5707963f, 0.f, 0.0825f, 0.f,    1.5707963f,  0.f,
                     -0.0825f, 0.384f, -1.5707963f, 0.f, 0.f,    0.f,    1.5707963f,  0.f,
                     0.088f,  0.f,    1.5707963f, 0.f};
  float lo[7] = {-2.8973f, -1.7628f, -2.8973f, -3.0718f, -2.8973f, -0.0175f, -2.8973f};
  float hi[7] = {2.8973f, 1.7628f, 2.8973f, -0.0698f, 2.8973f, 3.7525f, 2.8973f};
  float base[12];
  int32_t link[16];
  float xyzr[16 * 4];
  explicit Arm(float x, float yaw) {
    const float c = std::cos(yaw), s = std::sin(yaw);
    const float b[12] = {c, -s, 0.f, x, s, c, 0.f, 0.f, 0.f, 0.f, 1.f, 0.f};
    std::memcpy(base, b, sizeof base);
    for (int k = 0; k < 16; ++k) {
      link[k] = k / 2;
      xyzr[4 * k + 0] = 0.f;
      xyzr[4 * k + 1] = 0.f;
      xyzr[4 * k + 2] = (k % 2) ? 0.1f : 0.f;
      xyzr[4 * k + 3] = 0.08f - 0.003f * (float)k;
    }
  }
  mrpop_robot robot() const {
    return mrpop_robot{7, dh, lo, hi, base, 16, link, xyzr};
  }
};

void random_configs(Rng &g, const Arm &a, int n, int R, std::vector<float> &out) {
  out.resize((size_t)n * 7 * R);
  for (int i = 0; i < n; ++i)
    for (int r = 0; r < R; ++r)
      for (int j = 0; j < 7; ++j)
        out[((size_t)i * R + r) * 7 + j] = (float)(a.lo[j] + g.u() * (a.hi[j] - a.lo[j]));
}

template <class T>
T *to_device(const std::vector<T> &h) {
  T *d = nullptr;
  HIPCHECK(hipMalloc(&d, sizeof(T) * std::max<size_t>(1, h.size())));
  if (!h.empty()) HIPCHECK(hipMemcpy(d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice));
  return d;
}

mrpop_plan_params small_params(uint64_t seed) {
  mrpop_plan_params p;
  mrpop_plan_params_default(&p);
  p.seed = seed;
  p.candidates = 64;
  p.max_rounds = 60;
  p.max_iterations = 2;
  p.n_roadmap = 16;
  p.max_tree_nodes = 4096;
  p.max_roadmap_nodes = 1024;
  return p;
}

}  // namespace

int main() {
  std::printf("library %s\n", mrpop_version());
  mrpop_ctx *ctx = nullptr;
  CHECK(mrpop_ctx_create(0, &ctx) == MRPOP_OK);
  CHECK(mrpop_ctx_create(-1, nullptr) == MRPOP_E_INVALID_ARG);

  const Arm a0(-0.8f, 0.f), a1(0.8f, 3.14159265f);
  const mrpop_robot robots[2] = {a0.robot(), a1.robot()};
  const float spheres[2 * 4] = {0.f, 1.0f, 0.5f, 0.1f, 0.f, -1.1f, 0.9f, 0.1f};
  const float boxes[1 * 6] = {-0.1f, -1.3f, 0.2f, 0.1f, -1.1f, 0.4f};
  const mrpop_env env{2, spheres, 1, boxes};
  mrpop_scene *sc = nullptr;
  CHECK(mrpop_scene_create(ctx, robots, 2, &env, &sc) == MRPOP_OK);
  mrpop_scene *none_sc = nullptr;
  CHECK(mrpop_scene_create(ctx, robots, 0, &env, &none_sc) == MRPOP_E_INVALID_ARG && none_sc == nullptr);
  const int D = mrpop_scene_dof(sc);
  CHECK(D == 14 && mrpop_scene_total_spheres(sc) == 32);
  CHECK(mrpop_scene_set_tile_mode(sc, MRPOP_TILE_SCALAR) == MRPOP_OK);
  CHECK(mrpop_scene_tile_mode(sc) == MRPOP_TILE_SCALAR);
  CHECK(mrpop_scene_set_tile_mode(sc, 7) == MRPOP_E_INVALID_ARG);
  CHECK(mrpop_scene_set_tile_mode(sc, MRPOP_TILE_AUTO) == MRPOP_OK);

  // validation: the allocating and the allocation-free calls agree
  Rng g{0x9e3779b97f4a7c15ull};
  const int E = 500;
  std::vector<float> ha, hb;
  random_configs(g, a0, E, 2, ha);
  random_configs(g, a0, E, 2, hb);
  for (int e = 0; e < E; ++e)  // shorten the edges: a few to a few dozen states
    for (int j = 0; j < D; ++j) hb[(size_t)e * D + j] = ha[(size_t)e * D + j] + 0.1f * (hb[(size_t)e * D + j] - ha[(size_t)e * D + j]);
  float *qa = to_device(ha), *qb = to_device(hb);
  uint8_t *v1 = nullptr, *v2 = nullptr;
  HIPCHECK(hipMalloc(&v1, E));
  HIPCHECK(hipMalloc(&v2, E));
  CHECK(mrpop_profile_enable(ctx, -1) == MRPOP_E_INVALID_ARG);
  CHECK(mrpop_profile_enable(ctx, 1) == MRPOP_OK);
  mrpop_validate_stats vs{};
  CHECK(mrpop_validate_edges(ctx, sc, qa, qb, E, 0.05f, nullptr, v1, &vs, nullptr) == MRPOP_OK);
  CHECK(vs.edge_states > E);
  CHECK(mrpop_validate_edges_noalloc(ctx, sc, qa, qb, E, 0.05f, nullptr, v2, nullptr, nullptr) == MRPOP_OK);
  HIPCHECK(hipDeviceSynchronize());
  std::vector<uint8_t> b1(E), b2(E);
  HIPCHECK(hipMemcpy(b1.data(), v1, E, hipMemcpyDeviceToHost));
  HIPCHECK(hipMemcpy(b2.data(), v2, E, hipMemcpyDeviceToHost));
  CHECK(b1 == b2);
  CHECK(mrpop_validate_edges_noalloc(ctx, sc, qa, qb, MRPOP_NOALLOC_MAX_EDGES + 1, 0.05f, nullptr, v2, nullptr,
                                     nullptr) == MRPOP_E_INVALID_ARG);
  CHECK(mrpop_validate_edges(ctx, sc, qa, qb, E, -1.f, nullptr, v1, nullptr, nullptr) == MRPOP_E_INVALID_ARG);
  {  // caller-counted validation: every edge at its start state alone
    int32_t *dn = nullptr;
    HIPCHECK(hipMalloc(&dn, sizeof(int32_t) * (MRPOP_COUNTED_MAX_EDGES + 1)));
    std::vector<int32_t> ones(MRPOP_COUNTED_MAX_EDGES + 1, 1);
    HIPCHECK(hipMemcpy(dn, ones.data(), sizeof(int32_t) * ones.size(), hipMemcpyHostToDevice));
    CHECK(mrpop_validate_counted(ctx, sc, qa, qb, E, nullptr, v2, nullptr, nullptr) == MRPOP_E_INVALID_ARG);
    CHECK(mrpop_validate_counted(ctx, sc, qa, qb, MRPOP_COUNTED_MAX_EDGES + 1, dn, v2, nullptr, nullptr) ==
          MRPOP_E_INVALID_ARG);
    const int64_t nc = E < MRPOP_COUNTED_MAX_EDGES ? E : MRPOP_COUNTED_MAX_EDGES;
    mrpop_validate_stats cs{};
    CHECK(mrpop_validate_counted(ctx, sc, qa, qb, nc, dn, v2, &cs, nullptr) == MRPOP_OK);
    CHECK(cs.edge_states == nc);
    HIPCHECK(hipFree(dn));
  }
  mrpop_kernel_profile prof{};
  CHECK(mrpop_profile_read(ctx, &prof) == MRPOP_OK && prof.launches >= 1);
  CHECK(mrpop_profile_enable(ctx, 0) == MRPOP_OK);
  std::printf("validate: %lld edge states, %lld invalid edges\n", (long long)vs.edge_states,
              (long long)vs.edges_invalid);

  // a scene with many obstacles packed near the arms (per-link obstacle
  // lists, with the cluster level where the scene's estimate keeps it): the
  // same edges
  CHECK(mrpop_scene_obstacle_clusters(nullptr) == 0 && mrpop_scene_obstacle_clusters(sc) == 0);
  {
    std::vector<float> many_s, many_b;
    for (int k = 0; k < 90; ++k) {
      const float u = (float)g.u(), w = (float)g.u();
      many_s.insert(many_s.end(), {-0.2f + 0.4f * u, 1.0f + 0.3f * w, 0.3f + 0.4f * u * w, 0.02f});
    }
    for (int k = 0; k < 41; ++k) {
      const float u = (float)g.u(), w = (float)g.u();
      const float x = -0.2f + 0.4f * u, y = -1.3f + 0.3f * w, z = 0.3f + 0.3f * u * w;
      many_b.insert(many_b.end(), {x, y, z, x + 0.03f, y + 0.03f, z + 0.03f});
    }
    const mrpop_env env_many{90, many_s.data(), 41, many_b.data()};
    mrpop_scene *dense = nullptr;
    CHECK(mrpop_scene_create(ctx, robots, 2, &env_many, &dense) == MRPOP_OK);
    const int nc = mrpop_scene_obstacle_clusters(dense);
    CHECK(nc >= 0 && nc <= 2 * (MRPOP_MAX_JOINTS + 1) * ((90 + 41 + 7) / 8));
    CHECK(mrpop_validate_edges(ctx, dense, qa, qb, E, 0.05f, nullptr, v1, nullptr, nullptr) == MRPOP_OK);
    HIPCHECK(hipDeviceSynchronize());
    std::printf("dense scene: %d obstacle clusters\n", nc);
    mrpop_scene_destroy(dense);
  }

  // forward kinematics, nearest, sample
  float *xyzr = nullptr;
  HIPCHECK(hipMalloc(&xyzr, sizeof(float) * 16 * 32 * 4));
  CHECK(mrpop_fk_spheres(ctx, sc, qa, 16, xyzr, nullptr) == MRPOP_OK);
  int32_t *idx = nullptr;
  HIPCHECK(hipMalloc(&idx, sizeof(int32_t) * 32));
  CHECK(mrpop_nearest(ctx, qa, nullptr, E, D, qb, nullptr, 32, idx, nullptr) == MRPOP_OK);
  CHECK(mrpop_nearest(ctx, qa, nullptr, -1, D, qb, nullptr, 32, idx, nullptr) == MRPOP_E_INVALID_ARG);
  float *sq = nullptr, *scst = nullptr;
  HIPCHECK(hipMalloc(&sq, sizeof(float) * 32 * D));
  HIPCHECK(hipMalloc(&scst, sizeof(float) * 32));
  CHECK(mrpop_sample(ctx, sc, qa, qa + D, qa, 30.f, 1, 0, 0, 32, sq, scst, nullptr) == MRPOP_OK);
  HIPCHECK(hipDeviceSynchronize());

  // planning: plain, with history, rewiring, replanning; start and goal are
  // the first two free states among random ones (single-state edges)
  std::vector<float> cand;
  const int NC = 256;
  random_configs(g, a0, NC, 2, cand);
  float *dc = to_device(cand);
  uint8_t *vc = nullptr;
  HIPCHECK(hipMalloc(&vc, NC));
  CHECK(mrpop_validate_edges(ctx, sc, dc, dc, NC, 0.05f, nullptr, vc, nullptr, nullptr) == MRPOP_OK);
  HIPCHECK(hipDeviceSynchronize());
  std::vector<uint8_t> free_c(NC);
  HIPCHECK(hipMemcpy(free_c.data(), vc, NC, hipMemcpyDeviceToHost));
  std::vector<int> picks;
  for (int i = 0; i < NC && picks.size() < 2; ++i)
    if (free_c[i]) picks.push_back(i);
  CHECK(picks.size() == 2);
  std::vector<float> start(cand.begin() + (size_t)picks[0] * D, cand.begin() + (size_t)(picks[0] + 1) * D);
  std::vector<float> goal(cand.begin() + (size_t)picks[1] * D, cand.begin() + (size_t)(picks[1] + 1) * D);
  HIPCHECK(hipFree(dc));
  HIPCHECK(hipFree(vc));
  const int cap = 4096;
  std::vector<float> path((size_t)cap * D);
  int32_t len = 0;
  float cost = 0.f;
  mrpop_plan_stats st{};
  mrpop_plan_params p = small_params(1);
  const mrpop_status s_plan = mrpop_plan(ctx, sc, start.data(), goal.data(), &p, path.data(), cap, &len, &cost, &st);
  mrpop_status s = s_plan;
  std::printf("plan: status %d, %d waypoints, cost %.4f, %d rounds\n", (int)s, len, cost, st.rounds);
  CHECK(s == MRPOP_OK || s == MRPOP_E_NO_SOLUTION || s == MRPOP_E_START_INVALID || s == MRPOP_E_GOAL_INVALID);
  const bool solved = s == MRPOP_OK;
  std::vector<float> prev(path.begin(), path.begin() + (size_t)(solved ? len : 0) * D);

  std::vector<int32_t> offsets(17), rounds(16), vids((size_t)512 * 2);
  std::vector<float> hcost(16), wp((size_t)512 * D), rmv((size_t)2 * 256 * MRPOP_RM_STRIDE);
  std::vector<double> found(16);
  std::vector<int32_t> rme((size_t)2 * 512 * 2);
  mrpop_plan_history h;
  std::memset(&h, 0, sizeof h);
  h.entry_cap = 16;
  h.waypoint_cap = 512;
  h.offsets = offsets.data();
  h.costs = hcost.data();
  h.found_s = found.data();
  h.found_round = rounds.data();
  h.waypoints = wp.data();
  h.vertex_ids = vids.data();
  h.rm_vertices = rmv.data();
  h.rm_edges = rme.data();
  h.rm_vertex_cap = 256;
  h.rm_edge_cap = 512;
  s = mrpop_plan_with_history(ctx, sc, start.data(), goal.data(), &p, path.data(), cap, &len, &cost, &st, &h);
  std::printf("plan with history: status %d, %d entries\n", (int)s, h.n_entries);
  CHECK(s == MRPOP_OK || s == MRPOP_E_NO_SOLUTION || s == MRPOP_E_START_INVALID || s == MRPOP_E_GOAL_INVALID);

  mrpop_plan_params pr = small_params(2);
  pr.rewire = 1;
  s = mrpop_plan(ctx, sc, start.data(), goal.data(), &pr, path.data(), cap, &len, &cost, &st);
  std::printf("rewire plan: status %d, rewired %lld\n", (int)s, (long long)st.rewired);
  CHECK(s == MRPOP_OK || s == MRPOP_E_NO_SOLUTION || s == MRPOP_E_START_INVALID || s == MRPOP_E_GOAL_INVALID);
  pr.direct = 1;
  CHECK(mrpop_plan(ctx, sc, start.data(), goal.data(), &pr, path.data(), cap, &len, &cost, &st) ==
        MRPOP_E_INVALID_ARG);

  int32_t kept = -1;
  s = mrpop_replan(ctx, sc, start.data(), goal.data(), &p, solved ? prev.data() : nullptr,
                   solved ? (int32_t)(prev.size() / D) : 0, path.data(), cap, &len, &cost, &st, &kept);
  std::printf("replan: status %d, previous path kept %d\n", (int)s, kept);
  CHECK(kept == (solved ? 1 : 0));
  CHECK(mrpop_plan(ctx, sc, start.data(), goal.data(), &p, path.data(), 1, &len, &cost, &st) ==
        (solved ? MRPOP_E_BUFFER : s_plan));

  // a new environment, then a batch of three plans
  const float moved[4] = {0.f, 0.45f, 0.6f, 0.08f};
  const mrpop_env env2{1, moved, 0, nullptr};
  CHECK(mrpop_scene_set_env(sc, &env2) == MRPOP_OK);
  std::vector<std::vector<float>> bpaths(3, std::vector<float>((size_t)cap * D));
  mrpop_plan_request reqs[3];
  std::memset(reqs, 0, sizeof reqs);
  for (int i = 0; i < 3; ++i) {
    reqs[i].scene = sc;
    reqs[i].q_start = start.data();
    reqs[i].q_goal = goal.data();
    reqs[i].params = small_params(10 + i);
    reqs[i].path_out = bpaths[i].data();
    reqs[i].path_cap = cap;
  }
  mrpop_batch_stats bs{};
  CHECK(mrpop_plan_batch(ctx, reqs, 3, &bs) == MRPOP_OK);
  std::printf("batch: %d of %d solved, %lld launches\n", bs.solved, bs.instances, (long long)bs.launches);
  CHECK(mrpop_plan_batch(ctx, nullptr, 3, &bs) == MRPOP_E_INVALID_ARG);

  // serving
  mrpop_server *srv = nullptr;
  const mrpop_server_config cfg{2, 0};
  CHECK(mrpop_server_create(ctx, &cfg, &srv) == MRPOP_OK);
  int64_t tickets[4];
  for (int i = 0; i < 4; ++i) {
    const mrpop_plan_params q = small_params(20 + i);
    CHECK(mrpop_server_submit(srv, sc, start.data(), goal.data(), &q, &tickets[i]) == MRPOP_OK);
  }
  for (int i = 0; i < 4; ++i) {
    mrpop_server_result r{};
    CHECK(mrpop_server_wait(srv, tickets[i], 120.0, &r) == MRPOP_OK);
    CHECK(r.status != MRPOP_PENDING && r.t_submit <= r.t_admit && r.t_admit <= r.t_done);
    if (r.status == MRPOP_OK) CHECK(mrpop_server_path(srv, tickets[i], path.data(), cap) == MRPOP_OK);
    CHECK(mrpop_server_release(srv, tickets[i]) == MRPOP_OK);
  }
  mrpop_server_result none{};
  CHECK(mrpop_server_poll(srv, 12345, &none) == MRPOP_E_INVALID_ARG);
  mrpop_server_stats ss{};
  CHECK(mrpop_server_get_stats(srv, &ss) == MRPOP_OK && ss.completed == 4);
  CHECK(mrpop_server_clock(srv) >= 0.0);
  mrpop_server_destroy(srv);

  // the tuner's bookkeeping
  CHECK(mrpop_tuner_configure(nullptr, 0) == MRPOP_OK);
  std::printf("tuner entries %d\n", mrpop_tuner_entries());

  HIPCHECK(hipFree(qa));
  HIPCHECK(hipFree(qb));
  HIPCHECK(hipFree(v1));
  HIPCHECK(hipFree(v2));
  HIPCHECK(hipFree(xyzr));
  HIPCHECK(hipFree(idx));
  HIPCHECK(hipFree(sq));
  HIPCHECK(hipFree(scst));
  mrpop_scene_destroy(sc);
  mrpop_ctx_destroy(ctx);
  std::printf("host driver ok\n");
  return 0;
}
