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
  MRPOP_E_DEVICE = 9         /* a HIP runtime call failed                       */
} mrpop_status;

typedef struct mrpop_ctx mrpop_ctx;
typedef struct mrpop_scene mrpop_scene;

/* ------------------------------------------------------------------------ */
/* Context                                                                   */
/* ------------------------------------------------------------------------ */

/* Create a context bound to HIP device `device`.  The context owns the
 * library's device scratch (grown on demand, freed by destroy). */
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
void mrpop_scene_destroy(mrpop_scene *scene);
/* Composite dimension D (sum of joints) and total sphere count. */
int32_t mrpop_scene_dof(const mrpop_scene *scene);
int32_t mrpop_scene_total_spheres(const mrpop_scene *scene);

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
   * bounding spheres), exact link-box tests, coarse link-link tests, fine
   * sphere-sphere, sphere-box and arm-arm sphere tests. */
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

/* ------------------------------------------------------------------------ */
/* Kernel profiling                                                          */
/* ------------------------------------------------------------------------ */

/* Totals over the launches of the edge-validation tile kernel made on `ctx`
 * since profiling was (re-)enabled: launch count, summed kernel time taken
 * from HIP events recorded on the launch stream right before and after each
 * tile-kernel launch, and the states the kernel evaluated and was given. */
typedef struct {
  int64_t launches;
  double kernel_ms;
  int64_t states_checked;
  int64_t edge_states;
  int64_t work[8];        /* as mrpop_validate_stats.work, summed */
  int32_t grid_blocks;    /* workgroups of the last tile-kernel launch      */
  int32_t block_threads;  /* threads per workgroup                          */
} mrpop_kernel_profile;

/* enable != 0 starts recording (and clears the totals); 0 stops. */
mrpop_status mrpop_profile_enable(mrpop_ctx *ctx, int enable);
/* Waits for the recorded events and fills `out`.  E_INVALID_ARG if out is
 * NULL. */
mrpop_status mrpop_profile_read(mrpop_ctx *ctx, mrpop_kernel_profile *out);

#ifdef __cplusplus
}
#endif

#endif /* MRPOP_H */
