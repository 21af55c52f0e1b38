// Internal declarations of the planner kernels and their launchers.
#pragma once

#include "mrpop_internal.h"
#include "task.h"

namespace mrpop {

constexpr int kMaxDof = MRPOP_MAX_ROBOTS * MRPOP_MAX_JOINTS;
constexpr int kRmStride = MRPOP_RM_STRIDE;  // floats per roadmap vertex row (7 joints + pad)

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
  float *edge_a, *edge_b;     // [n][dim], or both null
  float res;                  // resolution of the edge's validation
  int32_t *n_codes;           // [n] or null: state-count code of each edge
  int direct;                 // 1: no roadmaps, steer toward q_rand by at most `step`
  float step;
};

// Device-side state of one search (a dRRT or AO-X call of Alg. 2): the tree
// the next round extends (the smaller one) and the trees' sizes, so that
// rounds can be queued back to back without the host deciding between them.
// The round that finds a connection or fills the tree sets `stop`; the rounds
// queued after it then do nothing.
struct SearchState {
  int32_t a;     // tree the next round extends: 0 is rooted at the start, 1 at the goal
  int32_t n[2];  // vertices per tree
  int32_t stop;
};

// Both search trees (structure of arrays), indexed by tree.
struct TreePair {
  float *q[2];       // [dim][tree_cap]
  float *g[2];       // [tree_cap]
  int32_t *vid[2];   // [n_robots][tree_cap]
  int32_t *parent[2];
  int32_t *n[2];     // vertex count (a copy of the search state's)
  float *e[2];       // [tree_cap] length of the edge to the parent (ao-dRRT), or null
};

constexpr int kMaxCandidates = 4096;  // candidates per round (mrpop_plan_params.candidates)

// ao-dRRT (the rewiring baseline of the paper's experiments): per candidate,
// the cheapest parent among the extended tree's tensor-product neighbours of
// q_new, and up to kRwSlots rewiring proposals (tree vertices whose cost
// drops through q_new, largest drop first, ties to the lower index).
constexpr int kRwSlots = 4;
constexpr int kRwMaxRoadmap = 8192;  // roadmap vertices per arm (LDS bitmap of a candidate's neighbours)
struct RewireArgs {
  int on;                  // 0: AO-X rounds; the fields below are not read
  int32_t *prop_z;         // [n][kRwSlots] proposal target in the extended tree, -1: none
  float *prop_cost;        // [n][kRwSlots] its cost through q_new
  float *prop_len;         // [n][kRwSlots] |q_new - q_z|
  float *edge_a, *edge_b;  // [n * kRwSlots][dim] proposal edges q_new -> q_z (null edges when unused)
  int32_t *n_codes;        // [n * kRwSlots] their state-count codes (0: unused slot)
  const uint8_t *pvalid;   // [n * kRwSlots] their validity (back half)
  float *e_new;            // [n] length of the extension edge (parent -> q_new)
  uint64_t *key;           // [tree_cap] scratch: the winning proposal per target (back half)
};

struct RoundStatus {
  int32_t found, cand, a_idx, b_idx;
  float total;
  int32_t inserted, overflow;
  int32_t a;        // the tree this round extended
  int32_t skipped;  // 1: the search had stopped before this round
  uint32_t seq;  // in the host copy: stored last, with a system-scope release (the round's number)
  int64_t states_ext, states_conn;
  int64_t states_spec;  // states of connection edges checked for candidates that were not inserted
  int64_t states_rw;    // states of rewiring edges (ao-dRRT)
  int32_t rewired;      // tree vertices that took a new parent (ao-dRRT)
  int32_t n_after;      // vertices of the extended tree after the round
};

struct ConnArgs {
  int n, dim;
  const int32_t *conn_idx;
  const float *q_new, *other_q;
  int tree_cap;
  float *edge_a, *edge_b;
  float res;          // resolution of the edge's validation
  int32_t *n_codes;   // [n] or null: state-count code of each edge
};

// The sample of each candidate and its nearest vertex in the extended tree
// (q.queries = s.out_q, q.budgets = s.out_c or null).
struct SampleNearArgs {
  SampleArgs s;
  NearestArgs q;
};

// The front half of a search round, one workgroup (256 threads) per
// candidate: the sample and its nearest vertex in the extended tree (sn), the
// extension (e: along the roadmaps, or a steer when e.direct; e.near_idx is
// sn.q's output), then, before the extension edge is known to be free, the
// connection: the budget c_best - g_new (-1 for a dead candidate: nothing is
// admissible), the nearest vertex of the other tree under it (q2: queries =
// e.q_new, budgets = budget) and the connection edge (c: conn_idx =
// q2.out_idx).  The extension edges and the connection edges are rows
// [0, n) and [n, 2n) of one batch, checked by one validation.
struct RoundFrontArgs {
  SampleNearArgs sn;
  ExtendArgs e;
  float c_best;
  float *budget;  // [n]
  NearestArgs q2;
  ConnArgs c;
  // The trees and the search state: the kernel takes the extended tree a and
  // the other tree from them (the tree fields and sizes in sn, e, q2 and c
  // are replaced); when the search has stopped it writes edges with no states.
  TreePair t;
  const SearchState *ss;
  // ao-dRRT: no budget in NEAREST and the extension (c_rand unused); the
  // extension edge starts at the cheapest neighbouring parent (e.near_idx and
  // e.g_new are replaced by it); proposals go to rw.  Proposal edges are rows
  // [2n, 2n + kRwSlots n) of the round's batch.
  RewireArgs rw;
};

// The back half, one workgroup: the survivors (alive, extension edge free)
// enter the extended tree in candidate order up to its capacity; among the
// inserted candidates whose connection edge is free, the one of least total
// cost g_new + |q_new - q_conn| + g_conn (ties: lowest candidate) is the
// round's result, written to the status record and, with the sequence
// number stored last, to status_out.
struct InsertSelectArgs {
  int n, dim, n_robots;
  const uint8_t *alive, *valid, *cvalid;  // valid: extension edges; cvalid: connection edges
  const float *q_new, *g_new;
  const int32_t *vid_new, *near_idx, *conn_idx;
  TreePair t;         // the round extends tree ss->a and connects to the other
  int tree_cap;
  SearchState *ss;    // read, then advanced: sizes, the next tree (the smaller), stop
  int32_t *ins_idx;
  const int32_t *codes_conn;  // [n] state-count codes of the connection edges
  const uint64_t *counters;   // the round's validation counters ([1]: states of both halves)
  RoundStatus *status;
  RoundStatus *status_out;    // or null: receives the finished record (e.g. pinned host memory)
  uint32_t seq;
  // ao-dRRT: after insertion and selection, the proposals of inserted
  // candidates whose edge is free are applied when cheaper than the target's
  // cost, the cheapest per target (ties: the earliest in candidate and slot
  // order), which is the result of applying them one by one in that order.
  RewireArgs rw;
};

// ao-dRRT, after the back half: when the round rewired any vertex, every
// vertex's cost is recomputed as the sum of the edge lengths along its parent
// chain (one thread per vertex).
struct RefreshArgs {
  TreePair t;
  const RoundStatus *status;  // the round's record (tree, vertex count, rewired count)
  int tree_cap;
};

struct PathArgs {
  int a_idx, b_idx, dim, tree_cap, cap;
  const int32_t *parent_a, *parent_b;
  const float *q_a, *q_b;
  float *out;
  int32_t *out_len;
  int n_robots;
  const int32_t *vid_a, *vid_b;  // SoA [n_robots][tree_cap]: each vertex's roadmap vertex per arm
  int32_t *out_vid;              // [cap][n_robots]
};

struct TreeRootArgs {
  float *tree_q, *tree_g;
  int32_t *tree_vid, *tree_parent, *tree_n;
  float *tree_e;  // or null
  int tree_cap;
  const float *q;
  int dim, n_robots, vid;
  SearchState *ss;  // or null: set to a fresh search (tree 0 next, both trees of one vertex)
};

struct RmSampleArgs {
  float *out;
  int n, nj;
  const float *lo, *hi;
  uint64_t key;
  int64_t j0;
  int32_t *codes;  // or null: [n] state-count code of each sample as a zero-length edge
  const int32_t *skip;  // or null: when *skip != 0 nothing is drawn and every code is 0 (no states)
};

struct RmAcceptArgs {
  const float *cand;
  const uint8_t *valid;
  int n, nj, need;
  float *V;
  int32_t *n_v;
  int cap;
  int32_t *taken;
  int32_t *parent;  // union-find parent of every roadmap vertex
  int32_t *zero2;   // or null: two counters set to zero first (the arm's pair counts)
  const int32_t *skip;  // or null: when *skip != 0 nothing is accepted (taken = 0)
};

struct RmPairsArgs {
  const float *V;
  int i0, i1, nj;
  float delta;
  int32_t *count;
  int cap;
  int32_t *pair_ids;
  float *qa, *qb;
  const int32_t *i1_dev;  // or null: i1 is lowered to *i1_dev (the vertex count on the device)
  float res;              // resolution of the pairs' validation (for codes)
  int32_t *codes;         // or null: [cap] state-count code of each written pair
};

struct RmUnionArgs {
  const int32_t *pair_ids;
  const uint8_t *valid;
  const int32_t *n_pairs;
  int max_pairs, n_v;
  int32_t *parent, *connected;
  int32_t *edges, *n_edges;  // or null: the valid pairs are appended to the edge list [cap_edges][2]
  int cap_edges;
  int32_t *connected_out;    // or null: a second copy of the connectivity flag (e.g. pinned host memory)
  const uint64_t *cnt;       // or null: the arm's validation counters [16], copied to cnt_out
  uint64_t *cnt_out;
};

struct RmBfsArgs {
  const int32_t *edges, *n_edges;
  int cap_edges, n_v;
  int32_t *rowptr, *col;
  int col_cap;
  int32_t *deg, *level, *connected;  // level null: adjacency only
};

// 32-bit fill and byte copy (device or mapped pinned host memory).
struct FillArgs {
  uint32_t *dst;
  uint32_t value;
  int64_t n;  // words
};

struct CopyArgs {
  void *dst;
  const void *src;
  int64_t bytes;
};

hipError_t launch_sample(const SampleArgs &a, hipStream_t s);
hipError_t launch_extend(const ExtendArgs &a, hipStream_t s);
hipError_t launch_nearest(const NearestArgs &a, hipStream_t s);
hipError_t launch_path(const PathArgs &a, hipStream_t s);
hipError_t launch_tree_root(const TreeRootArgs &a, hipStream_t s);
hipError_t launch_rm_sample(const RmSampleArgs &a, hipStream_t s);
hipError_t launch_rm_accept(const RmAcceptArgs &a, hipStream_t s);
hipError_t launch_rm_pairs(const RmPairsArgs &a, hipStream_t s);
hipError_t launch_rm_csr_bfs(const RmBfsArgs &a, hipStream_t s);
hipError_t launch_rm_union(const RmUnionArgs &a, hipStream_t s);
hipError_t launch_fill(const FillArgs &a, hipStream_t s);
hipError_t launch_copy(const CopyArgs &a, hipStream_t s);

// Key of an arm's roadmap sample stream.
uint64_t roadmap_key(uint64_t seed, uint64_t stream_a, uint64_t stream_b);

// The same kernels over many independent argument records at once (record
// blockIdx.y of the device array `args`; grid_x = the most blocks any record
// needs, records that need fewer leave early).
enum class Op : uint8_t {
  Sample, Nearest, Path, TreeRoot, RmSample, RmAccept, RmPairs, RmBfs, RmUnion, Fill, Copy, RoundFront,
  InsertSelect, Refresh, Validate
};
constexpr int kNumOps = 15;
constexpr int kUfMaxVertices = 32768;  // roadmap vertices per arm (union-find in LDS)

// Blocks one record needs (0: nothing to do).
int op_blocks(Op op, const void *args);
size_t op_args_bytes(Op op);
hipError_t launch_op(Op op, const void *args, hipStream_t s);
hipError_t launch_op_batch(Op op, const void *d_args, int count, int grid_x, hipStream_t s);
// n (1..kGroupMax) records of one kind, independent of each other, in one
// launch with the records passed by value (blockIdx.y selects the record).
constexpr int kGroupMax = 8;
hipError_t launch_op_group(Op op, const void *const *args, int n, hipStream_t s);

// A validation request of the planner: edges (qa[i], qb[i]) of one scene;
// bits to out[i]; the call's counters (the validation counter layout, [1] =
// edge states) to the caller's device array counters[16].
struct ValidateReq {
  const SceneDev *scene;  // host copy of the scene's device descriptor
  const float *qa, *qb;
  int64_t n;
  float res;
  uint8_t *out;
  uint64_t *counters;
  const int32_t *n_codes;  // device [n] or null: state-count codes written by the edges' producer
};

// One unit of device work of a planning instance.
struct Cmd {
  Op op;
  union {
    SampleArgs sample;
    NearestArgs nearest;
    PathArgs path;
    TreeRootArgs tree_root;
    RmSampleArgs rm_sample;
    RmAcceptArgs rm_accept;
    RmPairsArgs rm_pairs;
    RmBfsArgs rm_bfs;
    RmUnionArgs rm_union;
    FillArgs fill;
    CopyArgs copy;
    RoundFrontArgs round_front;
    InsertSelectArgs insert_select;
    RefreshArgs refresh;
    ValidateReq val;
  };
  const void *args() const { return &sample; }
};

// Where a planning instance's device work goes: launched at once on a
// stream (a plain plan), or queued and merged with other instances' work (a
// batch).  Work is executed in submission order; sync() returns once all of
// it has completed (host buffers written by copies are then valid).
class Exec {
 public:
  virtual ~Exec() = default;
  virtual hipError_t submit(const Cmd &c) = 0;
  // Commands none of which depends on another (no validations among them):
  // they may run in any order or concurrently, after everything submitted
  // before them and before everything submitted after them.
  virtual hipError_t submit_independent(const Cmd *cs, int n) {
    for (int i = 0; i < n; ++i) {
      const hipError_t e = submit(cs[i]);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  virtual hipError_t sync() = 0;
  // Waits until *flag == value, where the last submitted command stores
  // value there last, with a system-scope release (then everything submitted
  // before has completed).  The default synchronises.
  virtual hipError_t wait_flag(const uint32_t *flag, uint32_t value) {
    (void)flag;
    (void)value;
    return sync();
  }
  // A deferred executor never blocks: at a synchronisation point the job's
  // coroutine is parked (park) and resumed once the submitted work has
  // completed, with that work's status (resumed_status).
  virtual bool deferred() const { return false; }
  virtual void park(std::coroutine_handle<> h) { (void)h; }
  virtual hipError_t resumed_status() { return hipSuccess; }
};

// co_await SyncPoint{ex, flag, value}: everything submitted to ex has
// completed (flag null: ex.sync(); else ex.wait_flag(flag, value)); yields the
// HIP status.  Immediate on a blocking executor; parks the coroutine on a
// deferred one.
struct SyncPoint {
  Exec &ex;
  const uint32_t *flag = nullptr;
  uint32_t value = 0;
  hipError_t err = hipSuccess;
  bool await_ready() {
    if (ex.deferred()) return false;
    err = flag ? ex.wait_flag(flag, value) : ex.sync();
    return true;
  }
  void await_suspend(std::coroutine_handle<> h) { ex.park(h); }
  hipError_t await_resume() { return ex.deferred() ? ex.resumed_status() : err; }
};

}  // namespace mrpop
