/*
 * mrpop.h -- C ABI of the MI355X (gfx950) MR. POP hot-path library.
 *
 * MR. POP plans for K serial arms at once: a composite configuration
 * q = (q^1, ..., q^K) concatenates the arms' joint vectors, and the composite
 * free space excludes contact with the environment and between arms (paper,
 * Sec. "Problem Setup").  The planner grows per-arm roadmaps, searches their
 * tensor product with bidirectional dRRT, then keeps improving the path with
 * the AO-x meta-algorithm (Alg. 1, Alg. 2); collision checking of composite
 * edges dominates its run time (Sec. "Multi-Thread Reassignment for Collision
 * Checking").
 *
 * Conventions shared by every entry point
 *   - Floating point inputs and outputs are IEEE single precision.
 *   - "device" pointers are HIP device allocations on the context's device;
 *     "host" pointers are ordinary host memory.  Device buffers are owned by
 *     the caller and must stay alive until the work queued on `stream` ends.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Entry points that take a stream only queue work on it and return; they
 *     never synchronise unless a stats pointer is given.
 *   - Every entry point checks its host-side arguments before queuing any
 *     work and returns a status; no exception crosses the ABI.  After an
 *     error, mrpop_last_error() gives a message.
 *   - A context is used by one host thread at a time; its internal scratch is
 *     reused by consecutive calls, so calls on one context that are queued on
 *     different streams must not overlap in time.
 */
#ifndef MRPOP_H
#define MRPOP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MRPOP_MAX_JOINTS 7         /* joints per arm (links 0..7)            */
#define MRPOP_MAX_SPHERES 256      /* collision spheres per arm              */
#define MRPOP_MAX_ROBOTS 16        /* arms per scene                          */
#define MRPOP_MAX_ENV 65536        /* environment spheres and boxes, each    */
#define MRPOP_MAX_STATES_PER_EDGE (1 << 24)

typedef enum {
  MRPOP_OK = 0,
  MRPOP_E_INVALID_ARG = 1,   /* a host-side argument is out of range            */
  MRPOP_E_NONFINITE = 2,     /* a NaN or infinity in an input                   */
  MRPOP_E_START_INVALID = 3, /* the start state is in collision                 */
  MRPOP_E_GOAL_INVALID = 4,  /* the goal state is in collision                  */
  MRPOP_E_NO_SOLUTION = 5,   /* the budget ran out before any solution          */
  MRPOP_E_CAPACITY = 6,      /* a tree or roadmap reached its capacity          */
  MRPOP_E_NOMEM = 7,         /* a device allocation failed                      */
  MRPOP_E_BUFFER = 8,        /* an output buffer is too small                   */
  MRPOP_E_DEVICE = 9,        /* a HIP runtime call failed                       */
  MRPOP_PENDING = 10         /* a served request is queued or running           */
} mrpop_status;

typedef struct mrpop_ctx mrpop_ctx;
typedef struct mrpop_scene mrpop_scene;

/* ------------------------------------------------------------------------ */
/* Context                                                                   */
/* ------------------------------------------------------------------------ */

/* Create a context bound to HIP device `device`.  The context owns the
 * library's device scratch (grown on demand, freed by destroy).  It also
 * keeps the buffers of finished plans for later plans (at most 1 GiB of
 * device memory and 64 MiB of pinned host memory), so that a plan allocates
 * nothing per call once the pool is warm; destroy frees them. */
mrpop_status mrpop_ctx_create(int device, mrpop_ctx **out);
void mrpop_ctx_destroy(mrpop_ctx *ctx);
/* Message of the last failed call on `ctx` ("" if none).  Valid until the
 * next call on the same context.  NULL ctx gives the last creation error. */
const char *mrpop_last_error(const mrpop_ctx *ctx);
/* Library version string. */
const char *mrpop_version(void);

/* ------------------------------------------------------------------------ */
/* Scene: arms and environment                                               */
/* ------------------------------------------------------------------------ */

/* One serial arm.  Kinematics follow Craig's modified Denavit-Hartenberg
 * convention: row j of `dh` is (a_{j-1}, d_j, alpha_{j-1}, theta_off_j) and
 * frame j is T_j = T_{j-1} RotX(alpha_{j-1}) TransX(a_{j-1})
 * RotZ(q_j + theta_off_j) TransZ(d_j), with T_0 = base_tf.  Link 0 is fixed
 * to the base; link j >= 1 moves with joint j.  The arm's collision geometry
 * is a set of spheres, each attached to one link (paper: each arm is
 * approximated by spheres; Sec. "Multi-Thread Reassignment ..."). */
typedef struct {
  int32_t n_joints;            /* 1..MRPOP_MAX_JOINTS                       */
  const float *dh;             /* host [n_joints][4]                        */
  const float *q_lo;           /* host [n_joints] joint lower limits (rad)  */
  const float *q_hi;           /* host [n_joints] joint upper limits (rad)  */
  const float *base_tf;        /* host [12] row-major 3x4 world-from-base   */
  int32_t n_spheres;           /* 1..MRPOP_MAX_SPHERES                      */
  const int32_t *sphere_link;  /* host [n_spheres] link index 0..n_joints   */
  const float *sphere_xyzr;    /* host [n_spheres][4] link-local centre, r  */
} mrpop_robot;

/* Static obstacles: spheres and axis-aligned boxes (lo <= hi per axis). */
typedef struct {
  int32_t n_spheres;
  const float *spheres;        /* host [n_spheres][4] centre, radius >= 0   */
  int32_t n_boxes;
  const float *boxes;          /* host [n_boxes][6] lo xyz, hi xyz          */
} mrpop_env;

/* Copy arms and environment to the device and precompute the per-link
 * bounding ("coarse") spheres.  The host arrays may be freed on return.
 * Errors: E_INVALID_ARG (counts or link indices out of range, lo > hi),
 * E_NONFINITE, E_NOMEM. */
mrpop_status mrpop_scene_create(mrpop_ctx *ctx, const mrpop_robot *robots, int32_t n_robots,
                                const mrpop_env *env, mrpop_scene **out);
/* Frees the scene, with the one-arm sub-scenes that its first roadmap plan
 * built and kept for later plans.  No plan may be running on the scene. */
void mrpop_scene_destroy(mrpop_scene *scene);

/* Replace a scene's obstacles (paper, Sec. "Hardware Deployment": replanning
 * amid moving obstacles, one update per tick).  The arms stay; the
 * environment arrays, filter rows and arm-pair data are rebuilt from env as
 * mrpop_scene_create builds them, and the tile mode is kept.  No work that
 * uses the scene may be in flight: its old device copy is freed.  Errors as
 * mrpop_scene_create; on error the scene is unchanged. */
mrpop_status mrpop_scene_set_env(mrpop_scene *scene, const mrpop_env *env);
/* Composite dimension D (sum of joints) and total sphere count. */
int32_t mrpop_scene_dof(const mrpop_scene *scene);
int32_t mrpop_scene_total_spheres(const mrpop_scene *scene);
/* Obstacle clusters of the scene's coarse filter (performance only; the
 * bits do not depend on it).  Each link of each arm tests only the obstacles
 * within the link's reach of its arm's base, in Morton order of their
 * centres.  A list of 64 obstacles or more may group them in clusters of 8
 * with bounding spheres of their own, tested before their members; it keeps
 * them only when an estimate from the link's positions at random
 * configurations puts its coarse tests at half the list's length or less.
 * Returns the clusters over all lists, 0 when every list has one level (and
 * for a NULL scene). */
int32_t mrpop_scene_obstacle_clusters(const mrpop_scene *scene);

/* Where the edge-validation kernel reads the scene's coarse filter rows
 * (performance only; every mode gives the same bits):
 *   MRPOP_TILE_AUTO   -- LDS when the scene's copy fits the LDS budget
 *                        without lowering the workgroups a CU holds,
 *                        otherwise scalar loads (the default);
 *   MRPOP_TILE_LDS    -- a copy in LDS per workgroup (falls back to scalar
 *                        loads when it does not fit);
 *   MRPOP_TILE_SCALAR -- scalar loads from device memory.
 * Errors: E_INVALID_ARG (NULL scene or unknown mode). */
enum { MRPOP_TILE_AUTO = 0, MRPOP_TILE_LDS = 1, MRPOP_TILE_SCALAR = 2 };
mrpop_status mrpop_scene_set_tile_mode(mrpop_scene *scene, int32_t mode);
int32_t mrpop_scene_tile_mode(const mrpop_scene *scene);

/* ------------------------------------------------------------------------ */
/* Forward kinematics to world spheres                                       */
/* ------------------------------------------------------------------------ */

/* For each of n_cfg composite configurations q (device [n_cfg][D]), write
 * every arm's spheres in world coordinates to out_xyzr (device
 * [n_cfg][S_total][4]: x, y, z, radius), arms in scene order and each arm's
 * spheres in its input order.  Joint limits are not checked.
 * Errors: E_INVALID_ARG (n_cfg < 0, NULL buffers with n_cfg > 0). */
mrpop_status mrpop_fk_spheres(mrpop_ctx *ctx, const mrpop_scene *scene, const float *q, int64_t n_cfg,
                              float *out_xyzr, void *stream);

/* ------------------------------------------------------------------------ */
/* Composite edge validation                                                 */
/* ------------------------------------------------------------------------ */

typedef struct {
  int64_t edge_states;    /* sum over edges of their state count             */
  int64_t states_checked; /* states fully evaluated (early exit skips some)  */
  int64_t edges_invalid;  /* edges with out_valid == 0                       */
  int64_t nonfinite_edges;/* edges rejected for NaN/inf endpoints            */
  int64_t tiles;          /* work tiles processed                            */
  /* Work executed: kinematic chains (arm x state), coarse link centres
   * placed, coarse link-obstacle sphere tests (environment spheres and box
   * bounding spheres, of the obstacles within each link's reach only; for
   * lists with obstacle clusters, also the tests of the links against the
   * clusters, whose members are then tested only where the cluster's test
   * passes), exact link-box tests, coarse
   * link-link tests, fine sphere-sphere, sphere-box and arm-arm sphere
   * tests. */
  int64_t work[8];
} mrpop_validate_stats;

/* Decide for each composite edge (qa[e], qb[e]) whether the straight motion
 * between them is collision-free ("(q, q') in C^f", Alg. 2; the paper checks
 * an edge at discretised states, Sec. "Multi-Thread Reassignment ...").
 *
 *   qa, qb        device [n_edges][D] endpoints.
 *   resolution    > 0: the edge has n = 1 + ceil(Linf / resolution) states,
 *                 Linf = max_j |qb_j - qa_j| (single precision, correctly
 *                 rounded division; n = 1 when qa == qb); state k is
 *                 qa + (k / (n - 1)) (qb - qa), the last one exactly qb.
 *   n_states_opt  device [n_edges] or NULL: explicit state counts (>= 1)
 *                 that replace the rule above.
 *   out_valid     device [n_edges]: 1 if no state collides, else 0.
 *
 * A state collides when some arm sphere is closer than its radius sum to an
 * environment sphere, inside or closer than its radius to a box, or closer
 * than the radius sum to a sphere of another arm (touching is free).  Both
 * endpoints are checked.  Self-contact within one arm and joint limits are not
 * checked.  An edge with a NaN or infinite endpoint gets 0 and is counted in
 * stats.nonfinite_edges.  If stats_opt is not NULL the call waits for the
 * stream and fills it.  Errors: E_INVALID_ARG (n_edges < 0, resolution <= 0
 * without n_states_opt, more than MRPOP_MAX_STATES_PER_EDGE states per edge
 * found in the data: the edge is then reported invalid and counted as
 * non-finite), E_NOMEM, E_DEVICE. */
mrpop_status mrpop_validate_edges(mrpop_ctx *ctx, const mrpop_scene *scene, const float *qa, const float *qb,
                                  int64_t n_edges, float resolution, const int32_t *n_states_opt,
                                  uint8_t *out_valid, mrpop_validate_stats *stats_opt, void *stream);

/* Edge validation as mrpop_validate_edges for at most MRPOP_COUNTED_MAX_EDGES
 * edges whose state counts the caller has made (the n_states output of
 * mrpop_extend, or counts of its own), in one launch: the planner's round
 * batches take this path.  n_states is a device array [n_edges]: a count
 * n > 0 checks edge e at the n states of the paper's discretisation (Sec.
 * "Multi-Thread Reassignment for Collision Checking"; n = 1: q_a alone);
 * n <= 0 reports the edge invalid without checking it (mrpop_extend writes -1
 * for a non-finite endpoint and -2 for an edge of more than
 * MRPOP_MAX_STATES_PER_EDGE states; with stats_opt a -2 makes the call
 * return E_INVALID_ARG once the bits are written, as mrpop_validate_edges
 * does for such an edge, and -1 counts as a non-finite edge).  The bits equal those of
 * mrpop_validate_edges with the same counts; which states are evaluated
 * before an edge is found colliding may differ (stats_opt->states_checked).
 * qa, qb, n_states and out_valid are the caller's device buffers, layout as
 * mrpop_validate_edges.  Errors: E_INVALID_ARG (NULL ctx, scene, buffer or
 * n_states, n_edges < 0 or > MRPOP_COUNTED_MAX_EDGES; nothing is queued),
 * E_NOMEM, E_DEVICE. */
#define MRPOP_COUNTED_MAX_EDGES 1024
mrpop_status mrpop_validate_counted(mrpop_ctx *ctx, const mrpop_scene *scene, const float *qa, const float *qb,
                                    int64_t n_edges, const int32_t *n_states, uint8_t *out_valid,
                                    mrpop_validate_stats *stats_opt, void *stream);

/* mrpop_validate_edges for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and the same bits, with the working memory in
 * a fixed device array of 6 MiB that the library holds on every GPU it runs
 * on until the process ends, instead of the context's scratch.  The call
 * makes no device or pinned allocation and no free; the caller still owns
 * qa, qb, n_states_opt and out_valid.  Profiling events are not recorded.
 * Every call on one GPU shares that GPU's array, whichever context makes it:
 * calls whose work overlaps on one GPU (other streams, other threads,
 * other contexts) race and must be serialised by the caller.  Nothing in the
 * array needs clearing between calls (each launch writes every word it reads).
 * Arguments, layout and statuses as mrpop_validate_edges, plus
 * E_INVALID_ARG for n_edges > MRPOP_NOALLOC_MAX_EDGES (nothing is queued). */
#define MRPOP_NOALLOC_MAX_EDGES 65536
mrpop_status mrpop_validate_edges_noalloc(mrpop_ctx *ctx, const mrpop_scene *scene, const float *qa,
                                          const float *qb, int64_t n_edges, float resolution,
                                          const int32_t *n_states_opt, uint8_t *out_valid,
                                          mrpop_validate_stats *stats_opt, void *stream);

/* Tile shapes of the validation kernel (performance only; the bits never
 * depend on them) are measured: the first launch of each kind (launch path,
 * arms, spheres per arm, obstacles, batch-size bucket) runs the tile kernel
 * once per candidate shape (at most 4, 8 and 16 wavefronts per workgroup),
 * timed on its stream, which the call then waits for, and later launches of
 * that kind use the fastest.  mrpop_validate_edges_noalloc and launches under
 * graph capture never measure.  The choices are kept per process; with a
 * cache file they are also appended to it, one JSON object per line, and
 * loaded by later processes.
 *   cache_file  path of the cache file, or NULL for none; the file is read
 *               now (missing: empty) and the in-memory choices are replaced.
 *   enable      1: measure unseen kinds; 0: use known choices, else the
 *               built-in rule.
 * Defaults before the first call: MRPOP_TUNE_CACHE (the file) and
 * MRPOP_AUTOTUNE ("0" disables measuring).  Process-wide; not to be called
 * while validations run.  Errors: E_INVALID_ARG (enable not 0 or 1). */
mrpop_status mrpop_tuner_configure(const char *cache_file, int32_t enable);
/* Number of launch kinds with a chosen shape. */
int32_t mrpop_tuner_entries(void);

/* ------------------------------------------------------------------------ */
/* Search primitives                                                         */
/* ------------------------------------------------------------------------ */

/* Cost-bounded nearest vertex, NEAREST(V, q, c) of Alg. 2: for each query i,
 * among vertices v with costs[v] + |queries[i] - vertices[v]| < budgets[i],
 * the one of least Euclidean distance; equal distances go to the lower cost,
 * then to the lower index.  out_idx[i] = -1 when no vertex qualifies.
 *   vertices  device [n_vertices][dim] (row-major)
 *   costs     device [n_vertices] or NULL (all zero)
 *   queries   device [n_queries][dim]
 *   budgets   device [n_queries] or NULL (+infinity)
 *   out_idx   device [n_queries]
 * Errors: E_INVALID_ARG (negative counts, dim < 1 or above 112, NULL
 * buffers with non-zero counts). */
mrpop_status mrpop_nearest(mrpop_ctx *ctx, const float *vertices, const float *costs, int64_t n_vertices,
                           int32_t dim, const float *queries, const float *budgets, int64_t n_queries,
                           int32_t *out_idx, void *stream);

/* Candidate samples of one search round (INFORMED_SAMPLE and the cost
 * coordinate of Alg. 2).  Candidate i uses the random streams keyed by
 * (seed, purpose, round, first + i).  With c_best = +infinity, q is uniform in
 * the scene's joint limits and c = +infinity.  Otherwise q is uniform in the
 * prolate hyperspheroid with foci q_start, q_goal and transverse diameter
 * c_best (clamped onto the joint limits) and c ~ U[|q - root|, c_best].
 *   q_start, q_goal, root  device [D];  out_q device [n][D];
 *   out_c device [n] or NULL.
 * Errors: E_INVALID_ARG (n < 0, NULL buffers, c_best NaN or below
 * |q_goal - q_start| is allowed and collapses onto the segment). */
mrpop_status mrpop_sample(mrpop_ctx *ctx, const mrpop_scene *scene, const float *q_start, const float *q_goal,
                          const float *root, float c_best, uint64_t seed, uint64_t round, int64_t first, int64_t n,
                          float *out_q, float *out_c, void *stream);

/* Roadmap rows: joint j of vertex u of arm r at
 * rm_vertices[((r * rm_cap) + u) * MRPOP_RM_STRIDE + j]. */
#define MRPOP_RM_STRIDE 8

/* The extension step of one search round, ORACLE_AOX of Alg. 2 (paper, Sec.
 * "Converge to Global Optimality"; with no budget it is dRRT's oracle), for n
 * candidates.  Candidate i extends tree vertex z = near_idx[i] toward
 * q_rand[i] with budget c_rand[i].  Per arm r, with v the arm's roadmap
 * vertex in z, a neighbour u of v is admissible when moving arm r alone keeps
 * g_z + |u - v| < c_rand; among the admissible neighbours the arm takes the
 * one of largest cosine with q_rand^r - v (ties: lowest id) and stays when
 * none has a positive cosine.  If the composite move then reaches the
 * budget, moving arms go back to staying, least aligned first (ties: higher
 * arm index first), until g_z + |q_new - q_z| < c_rand.  The candidate is
 * alive when some arm moves.  Device buffers; D = the scene's dimension,
 * R = its arms; the call queues one launch on `stream` after waiting for
 * earlier work on it (it stages the arms' joint table in the context). */
typedef struct {
  int32_t n;                  /* candidates                                   */
  const int32_t *near_idx;    /* [n] tree vertex extended; -1: none (dead)    */
  const float *q_rand;        /* [n][D] samples                               */
  const float *c_rand;        /* [n] budgets, or NULL (all +infinity)         */
  const float *tree_q;        /* [D][tree_cap] tree configurations (SoA)      */
  const float *tree_g;        /* [tree_cap] cost-to-come                      */
  const int32_t *tree_vid;    /* [R][tree_cap] each arm's roadmap vertex      */
  int32_t tree_cap;
  const float *rm_vertices;   /* [R][rm_cap][MRPOP_RM_STRIDE] roadmap rows     */
  const int32_t *rm_rowptr;   /* [R][rm_cap + 1] adjacency rows (CSR)         */
  const int32_t *rm_col;      /* [R][col_cap] neighbour ids                   */
  int32_t rm_cap, col_cap;
  float resolution;           /* for n_states                                 */
  float *q_new;               /* out [n][D]: q_new (q_z when nothing moves)   */
  int32_t *vid_new;           /* out [R][n]: roadmap vertex per arm (-1: dead) */
  float *g_new;               /* out [n]: g_z + |q_new - q_z| (+inf: dead)    */
  uint8_t *alive;             /* out [n]                                      */
  float *edge_a, *edge_b;     /* out [n][D] or both NULL: the edge to check,  */
                              /* q_z -> q_new, or q_z -> q_z when not alive   */
  int32_t *n_states;          /* out [n] or NULL: that edge's state count at  */
                              /* `resolution` (as mrpop_validate_edges)       */
} mrpop_extend_batch;

/* Errors: E_INVALID_ARG (NULL batch or buffers, negative sizes, resolution
 * <= 0 with n_states), E_NOMEM, E_DEVICE. */
mrpop_status mrpop_extend(mrpop_ctx *ctx, const mrpop_scene *scene, const mrpop_extend_batch *batch,
                          void *stream);

/* ------------------------------------------------------------------------ */
/* Planning (Alg. 1)                                                         */
/* ------------------------------------------------------------------------ */

typedef struct {
  uint64_t seed;
  float delta;               /* roadmap connection radius (rad, per-arm joint space) */
  int32_t n_roadmap;         /* free samples added per arm per roadmap growth round */
  int32_t candidates;        /* P: candidate iterations per search round (1..4096) */
  float resolution;          /* edge discretisation (rad), > 0 */
  int32_t max_rounds;        /* search rounds over the whole call, > 0 */
  int32_t max_iterations;    /* outer iterations: roadmap growth, then one search once every arm is connected */
  int32_t max_growth_rounds; /* roadmap growth rounds per iteration */
  double time_budget_s;      /* wall-clock budget in seconds; 0 = none */
  int32_t max_tree_nodes;    /* vertices per search tree */
  int32_t max_roadmap_nodes; /* vertices per arm roadmap */
  int32_t stop_at_first;     /* 1: return after the first solution */
  float warm_cost;           /* incumbent cost to beat (+infinity: none) */
  /* Direct mode (paper, Sec. "Single-Robot Simulation Benchmarks &
   * Ablations": without roadmaps the search runs in the configuration space
   * itself, a bidirectional RRT-Connect-style search followed by AO-X):
   * 1 skips ROADMAP, and an extension moves from q_near toward q_rand by at
   * most `step` (Euclidean, rad) instead of along roadmap edges. */
  int32_t direct;
  float step;                /* direct mode: extension length, > 0 */
  /* The asymptotically optimal multi-robot baseline of the paper's
   * experiments (Sec. "Methodology": a bidirectional ao-dRRT that improves
   * paths by rewiring instead of AO-X): 1 keeps both trees across searches;
   * NEAREST and the dRRT extension take no cost bound; a new vertex's parent
   * is its cheapest tensor-product neighbour in the tree, and up to four tree
   * vertices whose cost drops through it are rewired to it (largest drop
   * first), when their edge is free, with the costs of their descendants
   * recomputed.  Samples, the connection and its budget c_best - g_new are
   * as in AO-X.  Requires direct 0 and max_roadmap_nodes <= 8192. */
  int32_t rewire;
} mrpop_plan_params;

typedef struct {
  double time_to_first_s;    /* wall time to the first solution, -1 if none */
  double total_time_s;
  int32_t rounds, iterations, solutions, first_round;
  int64_t edge_states;       /* composite edge states validated by the search:
                                the extension edges, and the connection edges of
                                the candidates that entered a tree */
  int64_t roadmap_edge_states;
  int32_t roadmap_vertices;  /* summed over arms */
  int32_t roadmap_connected; /* every arm's start and goal joined (last iteration) */
  int32_t capacity_hit;      /* a tree or roadmap reached its capacity */
  int32_t n_costs;           /* entries of costs[] */
  float costs[64];           /* incumbent cost after each improvement */
  /* Connection edges are searched and checked in the same launch as the
   * extension edges, before it is known which candidates enter the tree;
   * the states of those whose candidate did not (work done ahead and not
   * needed) are counted here and not in edge_states. */
  int64_t speculative_edge_states;
  int64_t rewired;           /* rewiring: tree vertices given a cheaper parent */
} mrpop_plan_stats;

/* Incumbent history (paper, Sec. "Seeding for Multi-Robot Jerk-Free
 * Motion": the paths found while the cost bound shrinks serve as seeds for a
 * local trajectory optimiser, cheaper paths first when there are more paths
 * than seeds).  Every host array is the caller's; mrpop_plan_with_history
 * writes the incumbents ranked by cost, cheapest first, as many as fit in
 * both entry_cap and waypoint_cap (the cheapest ones: a ranked prefix).
 *   waypoints    host [waypoint_cap][D]: the entries' paths back to back,
 *                each start to goal.
 *   offsets      host [entry_cap + 1]: entry k occupies rows
 *                offsets[k] .. offsets[k + 1] - 1.
 *   costs        host [entry_cap]: each entry's cost (sum of Euclidean
 *                waypoint steps, recomputed in double precision).
 *   found_s      host [entry_cap] or NULL: seconds from the call's start to
 *                the entry's discovery.
 *   found_round  host [entry_cap] or NULL: search round of the discovery.
 *   n_entries    out: incumbents found in the call (may exceed n_written).
 *   n_written    out: entries written.
 * Optional, for inspecting paths on the roadmaps' tensor product (Sec.
 * "Problem Setup": every edge of a path moves each arm along one of its
 * roadmap edges or keeps it in place, except that the connection of the two
 * trees is a straight composite edge):
 *   vertex_ids   host [waypoint_cap][R] or NULL: per written waypoint, each
 *                arm's roadmap vertex (meaningless in direct mode).
 *   rm_vertices  host [R][rm_vertex_cap][MRPOP_RM_STRIDE] or NULL: each arm's
 *                roadmap vertices at the end of the call (first
 *                rm_vertex_cap of them; vertex 0 is the arm's start, 1 its
 *                goal).
 *   rm_edges     host [R][rm_edge_cap][2] or NULL: each arm's roadmap edges
 *                (vertex pairs, first rm_edge_cap of them).
 *   rm_n_vertices, rm_n_edges  out: the full counts per arm (0 in direct
 *                mode). */
typedef struct {
  float *waypoints;
  int64_t waypoint_cap;
  int32_t *offsets;
  float *costs;
  double *found_s;
  int32_t *found_round;
  int32_t entry_cap;
  int32_t n_entries;
  int32_t n_written;
  int32_t *vertex_ids;
  float *rm_vertices;
  int32_t *rm_edges;
  int32_t rm_vertex_cap, rm_edge_cap;
  int32_t rm_n_vertices[MRPOP_MAX_ROBOTS];
  int32_t rm_n_edges[MRPOP_MAX_ROBOTS];
} mrpop_plan_history;

/* Defaults: seed 0, delta 3.0, n_roadmap 32, candidates 128, resolution
 * 0.05, max_rounds 1000, max_iterations 8, max_growth_rounds 16, no time
 * budget, 65536 tree and 8192 roadmap vertices, stop_at_first 0, no warm
 * cost, direct 0, step 1.0, rewire 0. */
void mrpop_plan_params_default(mrpop_plan_params *p);

/* MR. POP (Alg. 1): grow per-arm roadmaps (ROADMAP), search their tensor
 * product with bidirectional dRRT for a first path, then repeat roadmap
 * growth and cost-bounded search (AO-X) for strictly cheaper paths until a
 * budget runs out.  An iteration whose roadmaps leave some arm's start and
 * goal unconnected runs no search (the next one grows on); a search whose
 * tree fills up ends, and the next iteration starts afresh.  Blocking; runs
 * on the null stream of ctx's device.
 *   q_start, q_goal  host [D], composite configurations.
 *   path_out         host [path_cap][D]: the best path, start to goal.
 *   path_len         host: its number of waypoints (also on E_BUFFER).
 *   cost_out         host: its cost, the sum of Euclidean waypoint steps.
 *   stats_opt        host or NULL.
 * Status: OK with a path; E_START_INVALID / E_GOAL_INVALID when an endpoint
 * collides; E_NONFINITE; E_NO_SOLUTION when the budget ends without a path;
 * E_CAPACITY when the budget ends without a path after a search tree or a
 * roadmap filled up; E_BUFFER when path_cap is
 * too small; E_INVALID_ARG for out-of-range parameters. */
mrpop_status mrpop_plan(mrpop_ctx *ctx, const mrpop_scene *scene, const float *q_start, const float *q_goal,
                        const mrpop_plan_params *params, float *path_out, int32_t path_cap, int32_t *path_len,
                        float *cost_out, mrpop_plan_stats *stats_opt);

/* One replanning tick (paper, Sec. "Hardware Deployment": replanning amid
 * moving obstacles).  prev_path (host [prev_len][D]; NULL when prev_len is 0)
 * is the previous tick's path.  When it runs exactly from q_start to q_goal
 * and every one of its edges is free in the scene's current environment
 * (validated at params->resolution), it becomes the starting incumbent: the
 * call searches only for strictly cheaper paths (AO-X with c_best = its cost)
 * and returns it when none is found.  Otherwise the call plans from scratch.
 *   prev_valid_out  host or NULL: 1 when the previous path was kept.
 * Outputs and statuses as mrpop_plan. */
mrpop_status mrpop_replan(mrpop_ctx *ctx, const mrpop_scene *scene, const float *q_start, const float *q_goal,
                          const mrpop_plan_params *params, const float *prev_path, int32_t prev_len,
                          float *path_out, int32_t path_cap, int32_t *path_len, float *cost_out,
                          mrpop_plan_stats *stats_opt, int32_t *prev_valid_out);

/* mrpop_plan that also returns the incumbent history (above).  hist must not
 * be NULL; its arrays may be NULL only when entry_cap (offsets, costs) or
 * waypoint_cap (waypoints) is 0.  The plan's own status and outputs are those
 * of mrpop_plan; the history is written whenever the plan ran (also with
 * E_NO_SOLUTION, then empty). */
mrpop_status mrpop_plan_with_history(mrpop_ctx *ctx, const mrpop_scene *scene, const float *q_start,
                                     const float *q_goal, const mrpop_plan_params *params, float *path_out,
                                     int32_t path_cap, int32_t *path_len, float *cost_out,
                                     mrpop_plan_stats *stats_opt, mrpop_plan_history *hist);

/* ------------------------------------------------------------------------ */
/* Batched planning: many independent instances at once                     */
/* ------------------------------------------------------------------------ */

/* One planning instance of a batch.  Inputs as for mrpop_plan (host start,
 * goal and path buffer; the scene must come from the same context); the
 * outputs (status, path_len, cost, stats) are written by mrpop_plan_batch. */
typedef struct {
  const mrpop_scene *scene;
  const float *q_start, *q_goal;   /* host [D] */
  mrpop_plan_params params;
  float *path_out;                 /* host [path_cap][D] */
  int32_t path_cap;
  mrpop_status status;             /* out: as mrpop_plan would return */
  int32_t path_len;                /* out */
  float cost;                      /* out */
  mrpop_plan_stats stats;          /* out */
} mrpop_plan_request;

typedef struct {
  double wall_s;                   /* whole call */
  int32_t instances, solved;
  int64_t flushes;                 /* merged submissions of device work */
  int64_t launches;                /* kernel launches they made */
} mrpop_batch_stats;

/* Plans every request concurrently (the batching of the paper's many parallel
 * planning iterations, extended across independent problems): each instance
 * runs exactly the computation of mrpop_plan with the same parameters, so
 * with round/iteration budgets its path and cost equal the plain call's;
 * the device work of all instances is merged into shared launches, with the
 * edge validations of many scenes in one launch.  Wall-clock budgets
 * (time_budget_s) count from the start of the batch.  Returns E_INVALID_ARG
 * for a NULL context or request array; per-request failures are reported in
 * reqs[i].status.  Blocking; the instances run as coroutines on the calling
 * thread. */
mrpop_status mrpop_plan_batch(mrpop_ctx *ctx, mrpop_plan_request *reqs, int32_t n, mrpop_batch_stats *stats_opt);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of planning requests                         */
/* ------------------------------------------------------------------------ */

/* A server plans requests as they arrive.  A request waits in a queue until a
 * slot is free and its device memory (PlanJob arena and one-arm sub-scenes,
 * estimated before allocation) fits the budget next to the running ones; it
 * then runs alongside them, its device work merged with theirs at every
 * synchronisation point (as in mrpop_plan_batch), and its trees and roadmaps
 * stay on the device until it ends.  Each request computes exactly what
 * mrpop_plan computes for it alone (with round budgets; a time budget counts
 * from the request's admission). */
typedef struct mrpop_server mrpop_server;

typedef struct {
  int32_t max_slots;           /* requests running at once (1 .. 4096)        */
  int64_t mem_budget_bytes;    /* device memory for running requests (0: none) */
} mrpop_server_config;

typedef struct {
  mrpop_status status;         /* MRPOP_PENDING until the request ends        */
  int32_t path_len;
  float cost;
  mrpop_plan_stats stats;
  double t_submit, t_admit, t_done;  /* server clock (mrpop_server_clock), s  */
  int64_t device_bytes;        /* memory reserved for the request             */
} mrpop_server_result;

typedef struct {
  int64_t submitted, admitted, completed, rejected;
  int32_t queue_len, running, max_queue_len, max_running;
  int64_t reserved_bytes, peak_reserved_bytes;
  int64_t flushes, launches;
} mrpop_server_stats;

/* Starts the server's scheduling thread.  E_INVALID_ARG for a bad config.
 * The server uses the context (and the scenes of its requests) from that
 * thread until it is destroyed: meanwhile, only the mrpop_server_* calls may
 * be made on them. */
mrpop_status mrpop_server_create(mrpop_ctx *ctx, const mrpop_server_config *cfg, mrpop_server **out);
/* Finishes running requests, drops queued ones (they stay PENDING) and stops. */
void mrpop_server_destroy(mrpop_server *srv);
/* Queues a request.  Start, goal and params are copied; the scene must stay
 * alive until the request ends.  *ticket identifies it.  A request whose
 * memory exceeds the whole budget ends at once with E_NOMEM. */
mrpop_status mrpop_server_submit(mrpop_server *srv, const mrpop_scene *scene, const float *q_start,
                                 const float *q_goal, const mrpop_plan_params *params, int64_t *ticket);
/* Result of a request (status MRPOP_PENDING while it has not ended).  Returns
 * E_INVALID_ARG for an unknown ticket, MRPOP_OK otherwise. */
mrpop_status mrpop_server_poll(mrpop_server *srv, int64_t ticket, mrpop_server_result *out);
/* As poll, after waiting up to timeout_s seconds for the request to end. */
mrpop_status mrpop_server_wait(mrpop_server *srv, int64_t ticket, double timeout_s, mrpop_server_result *out);
/* Copies an ended request's path (start -> goal, [path_len][D]); E_BUFFER if
 * cap is too small, E_INVALID_ARG if the ticket is unknown or has no path. */
mrpop_status mrpop_server_path(mrpop_server *srv, int64_t ticket, float *path_out, int32_t cap);
/* Forgets an ended request's result. */
mrpop_status mrpop_server_release(mrpop_server *srv, int64_t ticket);
mrpop_status mrpop_server_get_stats(mrpop_server *srv, mrpop_server_stats *out);
/* Seconds on the server's clock (the clock of the result timestamps). */
double mrpop_server_clock(const mrpop_server *srv);

/* ------------------------------------------------------------------------ */
/* Kernel profiling                                                          */
/* ------------------------------------------------------------------------ */

/* Totals over the launches of the edge-validation tile kernel made on `ctx`
 * since profiling was (re-)enabled: launch count, summed kernel time taken
 * from HIP events recorded on the launch stream right before and after each
 * timed tile-kernel launch (every launch, or every k-th: see
 * mrpop_profile_enable), and the states the kernel evaluated and was given
 * (over every launch). */
typedef struct {
  int64_t launches;
  double kernel_ms;
  int64_t states_checked;
  int64_t edge_states;
  int64_t work[8];        /* as mrpop_validate_stats.work, summed */
  int32_t grid_blocks;    /* workgroups of the last tile-kernel launch      */
  int32_t block_threads;  /* threads per workgroup                          */
  int64_t timed_launches; /* launches whose time kernel_ms sums             */
} mrpop_kernel_profile;

/* enable != 0 starts recording (and clears the totals); 0 stops.  enable = 1
 * times every tile-kernel launch; enable = k > 1 times the first launch and
 * then every k-th (the event pair adds dispatch time to the launches it
 * brackets, so a sample keeps that cost off the others); the work totals
 * always cover every launch.  E_INVALID_ARG if enable < 0. */
mrpop_status mrpop_profile_enable(mrpop_ctx *ctx, int enable);
/* Waits for the recorded events and fills `out`.  E_INVALID_ARG if out is
 * NULL. */
mrpop_status mrpop_profile_read(mrpop_ctx *ctx, mrpop_kernel_profile *out);

#ifdef __cplusplus
}
#endif

#endif /* MRPOP_H */
