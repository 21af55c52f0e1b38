// One planning instance (Alg. 1 with the subroutines of Alg. 2) whose device
// work goes through an Exec, so that the same code runs a plain plan or one
// instance of a batch.
#pragma once

#include <string>
#include <vector>

#include "planner.h"

namespace mrpop {

class PlanJob {
 public:
  PlanJob() = default;
  PlanJob(const PlanJob &) = delete;
  PlanJob &operator=(const PlanJob &) = delete;
  ~PlanJob();

  // Host-side preparation: argument checks, device and pinned allocations,
  // the one-arm sub-scenes of the roadmaps.  Queues no device work.
  mrpop_status prepare(mrpop_ctx *ctx, const mrpop_scene *scene, const float *q_start, const float *q_goal,
                       const mrpop_plan_params &params);
  // The planner as a coroutine: every device operation goes through ex, and
  // every wait for device work is a suspension point (see SyncPoint).  On a
  // blocking executor one resume() runs it to the end (run_blocking).
  Task<mrpop_status> run(Exec &ex);
  mrpop_status run_blocking(Exec &ex);
  // Before run: a known collision-free path (start to goal, [len][D]) as the
  // incumbent to improve on; it is returned if no cheaper path is found.
  void set_incumbent(const std::vector<float> &path);

  // Results (after run): the best path (start -> goal, row-major [len][D]),
  // its cost recomputed in double precision, statistics, and the message of
  // a failed status.
  const std::vector<float> &path() const { return best_path_; }
  float cost() const { return c_best_; }
  const mrpop_plan_stats &stats() const { return st_; }
  const std::string &error() const { return err_; }
  // Every incumbent of the call in discovery order (strictly decreasing cost).
  struct Incumbent {
    std::vector<float> path;    // [len][D], start to goal
    std::vector<int32_t> vids;  // [len][R]: each waypoint's roadmap vertex per arm (-1: unknown)
    float cost;
    double found_s;
    int32_t round;
  };
  const std::vector<Incumbent> &history() const { return history_; }
  int dof() const { return D_; }
  int n_robots() const { return R_; }
  // After run: each arm's roadmap (vertex rows [rm_cap][kRmStride] and edge
  // list [edge_cap][2], at most the given capacities) into host arrays, and
  // the full counts; waits for the copies.
  mrpop_status export_roadmaps(float *V, int32_t v_cap, int32_t *E, int32_t e_cap, int32_t *n_v, int32_t *n_e);
  // Device bytes held by the instance (arena and sub-scenes).
  size_t device_bytes() const { return device_bytes_; }
  // Device bytes an instance of `scene` with `params` would hold (an upper
  // bound: the sub-scenes are counted at the size of the whole scene).
  static size_t device_bytes_for(const mrpop_scene *scene, const mrpop_plan_params &params);

 private:
  mrpop_status fail_(mrpop_status s, const std::string &m) {
    err_ = m;
    return s;
  }
  mrpop_status hip_fail_(hipError_t e, const char *what) {
    err_ = std::string(what) + ": " + hipGetErrorString(e);
    return MRPOP_E_DEVICE;
  }
  // n_codes (device, optional): state-count codes the edges' producer wrote
  mrpop_status validate_(Exec &ex, const mrpop_scene *sc, const float *a, const float *b, int64_t n, float res,
                         uint8_t *out, uint64_t *counters, const int32_t *n_codes = nullptr);
  mrpop_status copy_(Exec &ex, void *dst, const void *src, size_t bytes);
  // Submits cs as one group of independent commands, then clears it.
  mrpop_status group_(Exec &ex, std::vector<Cmd> &cs);
  Task<mrpop_status> roadmap_(Exec &ex, int it);
  // One sampling pass of growth round g (ROADMAP): samples of the arms in
  // `act` from stream position j0, their validation, acceptance and the pair
  // counts of the arms in `counted`, then the counts to pinned memory.  With
  // `speculative`, an arm whose connected flag is set on the device by then
  // draws and accepts nothing.
  mrpop_status rm_pass_(Exec &ex, int it, int g, int64_t j0, const std::vector<int> &act,
                        const std::vector<int> &counted, bool speculative, const std::vector<int> &need,
                        const std::vector<int> &n0, const std::vector<int> &need0);
  void set_sizes_(const mrpop_scene *scene, const mrpop_plan_params &P);
  size_t plan_arena_(void *base);  // assigns the arena's arrays (base may be null); returns its size
  double elapsed_() const;
  bool out_of_time_() const;

  mrpop_ctx *ctx_ = nullptr;
  const mrpop_scene *scene_ = nullptr;
  mrpop_plan_params P_{};
  int R_ = 0, D_ = 0, PC_ = 0, max_nj_ = 0;
  int rm_cap_ = 0, edge_cap_ = 0, col_cap_ = 0, cand_batch_ = 0, pair_cap_ = 0, tcap_ = 0, path_max_ = 0;
  double t_start_ = 0.0;
  std::string err_;
  mrpop_plan_stats st_{};
  float c_best_ = INFINITY;
  std::vector<float> best_path_;
  std::vector<Incumbent> history_;
  std::vector<int32_t> h_qoff_, h_nj_, rm_n_;
  std::vector<mrpop_scene *> arms_;  // the scene's cached one-arm sub-scenes (not owned)
  size_t device_bytes_ = 0;

  // device arena
  void *arena_ = nullptr;
  float *qs_, *qg_, *rm_V_, *cand_, *pair_qa_, *pair_qb_, *tq_[2], *tg_[2], *q_rand_, *c_rand_, *q_new_, *g_new_,
      *ea_, *eb_, *budget_, *ca_, *cb_, *path_d_;
  int32_t *path_vid_d_;  // [path_max][R] roadmap vertices of the extracted path
  // per arm r: cand_ [r][cand_batch][kRmStride], cand_valid_ and cand_codes_ [r][cand_batch],
  // rm_i_ [r][kRmInts] (taken, pair count, pair count when writing,
  // connected), uf_ [r][rm_cap] union-find parents, cnt_ [2 + r][16]
  int32_t *rm_rowptr_, *rm_col_, *rm_edges_, *rm_nv_, *rm_ne_, *pair_ids_, *rm_i_, *uf_, *deg_, *tvid_[2],
      *tpar_[2], *tn_[2], *near_idx_, *vid_new_, *ins_idx_, *conn_idx_, *d_nj_, *d_qoff_,
      *cand_codes_, *pair_codes_;
  int32_t *codes_ext_, *codes_conn_;  // [rows] state-count codes of the round's batch; codes_conn_ = codes_ext_ + PC
  // ao-dRRT: edge lengths to the parents [2][tree_cap], the proposals
  // [PC][kRwSlots] (their edges are rows [2 PC, 2 PC + kRwSlots PC) of the
  // round's batch), extension edge lengths [PC], the per-target key [tree_cap]
  float *te_[2] = {nullptr, nullptr}, *prop_cost_ = nullptr, *prop_len_ = nullptr, *e_new_ = nullptr;
  int32_t *prop_z_ = nullptr;
  uint64_t *rw_key_ = nullptr;
  int64_t batch_rows_ = 0;  // rows of a round's edge batch: 2 PC, plus kRwSlots PC with rewiring
  uint8_t *cand_valid_, *pair_valid_, *alive_, *valid_, *cvalid_;
  uint64_t *cnt_;  // [2 + R][16]: counters of the extension, connection and per-arm roadmap validations
  RoundStatus *status_;
  SearchState *ss_;   // the current search's state (device)
  uint32_t seq_ = 0;  // sequence number of the last round record queued
  static constexpr int kRmInts = 4;
  // Search rounds queued per host wait.  Rounds queued after the one that
  // connects do nothing (a launch each of the three kernels, a few us).
  static constexpr int kRoundsPerWait = 6;

  // pinned host memory (device-visible): uploads, and what comes back
  struct Pinned {
    RoundStatus status[kRoundsPerWait];  // the records of the queued rounds
    int32_t ints[4];
    uint8_t valid2[8];
  };
  Pinned *pin_ = nullptr;
  void *host_block_ = nullptr;  // pin_, pin_rm_, pin_cnt_, upload_, upload_i_ (one pooled pinned block)
  size_t arena_got_ = 0, host_got_ = 0;
  bool synced_ = true;  // false while run() may have queued work not yet waited for
  int32_t *pin_rm_ = nullptr;   // [R][kRmInts] copy of rm_i_, then [R] vertex counts
  uint64_t *pin_cnt_ = nullptr; // [R][16] copy of the arms' validation counters
  float *upload_ = nullptr;  // qs, qg, roadmap seeds [R][2][kRmStride]
  int32_t *upload_i_ = nullptr;  // nj, q_off
  float *pin_path_ = nullptr;
  size_t pin_path_cap_ = 0;
};

}  // namespace mrpop
