// Internal declarations of the planner kernels and their launchers.
#pragma once

#include "mrpop_internal.h"

namespace mrpop {

constexpr int kMaxDof = MRPOP_MAX_ROBOTS * MRPOP_MAX_JOINTS;
constexpr int kRmStride = 8;  // floats per roadmap vertex row (7 joints + pad)

// Purposes of the counter-based random streams.
constexpr uint64_t kPurposeQ = 1, kPurposeBall = 2, kPurposeC = 3, kPurposeRoadmap = 4;

struct SampleArgs {
  int n, dim;
  float c_best;
  uint64_t seed, round;
  int first;                  // stream index of candidate 0
  const float *lo, *hi;       // [dim] joint limits
  const float *qs, *qg;       // [dim] foci
  const float *root;          // lower-bound root; element j at root[j * root_stride]
  int64_t root_stride;
  float *out_q;               // [n][dim]
  float *out_c;               // [n] or null
};

struct NearestArgs {
  const float *V;             // vertex v, dimension j at V[v * v_stride + j * d_stride]
  const float *g;             // [n] cost-to-come or null (zeros)
  int64_t n;
  int dim;
  int64_t v_stride, d_stride;
  const float *queries;       // query i at queries[i * q_stride + j]
  int64_t q_stride;
  const float *budgets;       // [n_queries] or null (+inf)
  int64_t n_queries;
  int32_t *out_idx;           // [n_queries], -1 when no vertex is admissible
};

struct ExtendArgs {
  int n, dim, n_robots;
  const int32_t *near_idx;    // [n]
  const float *q_rand;        // [n][dim]
  const float *c_rand;        // [n] or null
  const float *tree_q;        // SoA [dim][tree_cap]
  const int32_t *tree_vid;    // SoA [R][tree_cap]
  const float *tree_g;
  int tree_cap;
  const float *rm_V;          // [R][rm_cap][kRmStride]
  const int32_t *rm_rowptr;   // [R][rm_cap + 1]
  const int32_t *rm_col;      // [R][rm_col_cap]
  int rm_cap, rm_col_cap;
  const int32_t *nj, *q_off;  // [R]
  float *q_new;               // [n][dim]
  int32_t *vid_new;           // [R][n]
  float *g_new;               // [n]
  uint8_t *alive;             // [n]
  float *edge_a, *edge_b;     // [n][dim]
};

struct RoundStatus {
  int32_t found, cand, a_idx, b_idx;
  float total;
  int32_t inserted, overflow, pad;
  int64_t states_ext, states_conn;
};

struct InsertArgs {
  int n, dim, n_robots;
  const uint8_t *alive, *valid;
  const float *q_new, *g_new;
  const int32_t *vid_new, *near_idx;
  float *tree_q, *tree_g;
  int32_t *tree_vid, *tree_parent, *tree_n;
  int tree_cap;
  float c_best;
  int32_t *ins_idx;
  float *budget;
  RoundStatus *status;
};

struct ConnArgs {
  int n, dim;
  const int32_t *conn_idx;
  const float *q_new, *other_q;
  int tree_cap;
  float *edge_a, *edge_b;
};

struct SelectArgs {
  int n, dim;
  const int32_t *ins_idx, *conn_idx;
  const uint8_t *cvalid;
  const float *q_new, *g_new, *other_q, *other_g;
  int tree_cap;
  const uint64_t *states_ext, *states_conn;  // validation counters (index 1: edge states)
  RoundStatus *status;
};

struct PathArgs {
  int a_idx, b_idx, dim, tree_cap, cap;
  const int32_t *parent_a, *parent_b;
  const float *q_a, *q_b;
  float *out;
  int32_t *out_len;
};

hipError_t launch_sample(const SampleArgs &a, hipStream_t s);
hipError_t launch_nearest(const NearestArgs &a, hipStream_t s);
hipError_t launch_extend(const ExtendArgs &a, hipStream_t s);
hipError_t launch_insert(const InsertArgs &a, hipStream_t s);
hipError_t launch_conn_edges(const ConnArgs &a, hipStream_t s);
hipError_t launch_select(const SelectArgs &a, hipStream_t s);
hipError_t launch_path(const PathArgs &a, hipStream_t s);
hipError_t launch_tree_root(float *tree_q, int32_t *tree_vid, float *tree_g, int32_t *tree_parent, int32_t *tree_n,
                            int tree_cap, const float *q, int dim, int n_robots, int vid, hipStream_t s);
hipError_t launch_rm_sample(float *out, int n, int nj, const float *lo, const float *hi, uint64_t seed,
                            uint64_t stream_a, uint64_t stream_b, int64_t j0, hipStream_t s);
hipError_t launch_rm_accept(const float *cand, const uint8_t *valid, int n, int nj, int need, float *V, int32_t *n_v,
                            int cap, int32_t *taken, hipStream_t s);
hipError_t launch_rm_pairs(const float *V, int i0, int i1, int nj, float delta, int32_t *count, int cap,
                           int32_t *pair_ids, float *qa, float *qb, hipStream_t s);
hipError_t launch_rm_add_edges(const int32_t *pair_ids, const uint8_t *valid, const int32_t *n_pairs, int max_pairs,
                               int32_t *edges, int32_t *n_edges, int cap_edges, hipStream_t s);
hipError_t launch_rm_csr_bfs(const int32_t *edges, const int32_t *n_edges, int cap_edges, int n_v, int32_t *rowptr,
                             int32_t *col, int col_cap, int32_t *deg, int32_t *level, int32_t *connected,
                             hipStream_t s);

}  // namespace mrpop
