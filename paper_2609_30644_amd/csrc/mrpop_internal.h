// Internal declarations of the MR. POP HIP library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "mrpop.h"

namespace mrpop {

constexpr int kMaxJoints = MRPOP_MAX_JOINTS;
constexpr int kMaxLinks = MRPOP_MAX_JOINTS + 1;
constexpr int kWave = 64;
constexpr int kClusterSize = 8;  // table rows per obstacle cluster of the coarse filter

// Device-side view of a scene, passed to kernels by value.
//
// Arms share one kinematic model when the scene is homogeneous (the common
// case: a team of identical arms); the kernels then read every model field
// with wave-uniform addresses (scalar loads).  Otherwise each arm carries its
// own model and the same fields are read per lane.
struct SceneDev {
  int32_t n_robots;
  int32_t dof;
  int32_t homogeneous;     // 1 if every arm uses model 0
  int32_t total_spheres;
  // per arm
  const int32_t *model;    // [R] model index
  const int32_t *q_off;    // [R] offset of the arm's joints in q
  const int32_t *s_out;    // [R] offset of the arm's spheres in FK output order
  const float *base;       // [R][12] world-from-base (recentred world frame)
  // per model (stride kMaxLinks / kMaxJoints / max spheres)
  int32_t n_models;
  int32_t sph_stride;      // spheres per model slot (max over models)
  const int32_t *nj;       // [M]
  const float4 *dh;        // [M][kMaxJoints]: a, d, cos(alpha), sin(alpha)
  const float *theta_off;  // [M][kMaxJoints]
  const int32_t *link_start;  // [M][kMaxLinks + 1] fine spheres grouped by link
  const int32_t *link_order;  // [M][kMaxLinks] links by decreasing sphere count (ties: lower link first)
  const float4 *fine;      // [M][sph_stride] link-local x, y, z, r (grouped by link)
  const int32_t *fine_src; // [M][sph_stride] index of the sphere in the input order
  const float4 *coarse;    // [M][kMaxLinks] link-local centre, radius (r < 0: empty link)
  // environment
  int32_t n_env_spheres;
  int32_t n_env_boxes;
  const float4 *env_s;     // [Ns] x, y, z, r (recentred)
  const float4 *env_b;     // [Nb][2] (lo x, lo y, lo z, 0), (hi x, hi y, hi z, 0) (recentred)
  float3 origin;           // world = recentred + origin
  // Coarse filter rows in expanded form, one list per (arm, link).  The
  // coarse sphere (centre c, radius rc) can touch an obstacle's bounding
  // sphere (centre o, radius s) only if
  //   |c|^2 - 2 c.o + |o|^2 - (rc + s + delta)^2 < 0,
  // so a row holds (-2 o_x, -2 o_y, -2 o_z, w) with w = |o|^2 - (rc + s +
  // delta)^2: each test is three FMAs from |c|^2 and a compare against -w.
  // delta bounds the single-precision error of the expanded form over the
  // scene's extent, so the filter never drops a contact.  A list holds only
  // the obstacles within the link's reach of its arm's base (the others can
  // never be touched), padded with never-passing rows (w = +3e38) to a
  // multiple of eight, as the kernel reads them in pairs of groups of four;
  // one more group of padding follows the last list.  row_obs gives each
  // row's obstacle: k < n_env_spheres is sphere k, otherwise box
  // k - n_env_spheres.
  // Lists of many obstacles may also have a cluster level: cluster c covers
  // rows kClusterSize c onwards, and its row holds the same expanded test for
  // a sphere containing every member's bounding sphere (with its own delta),
  // so a link that touches a member obstacle passes the cluster's test.
  // link_lists[r][l] = {row offset, rows (padded), obstacles, cluster-row
  // offset, cluster rows (padded), clusters (0: one level), 0, 0}.
  const int32_t *link_lists;  // [R][kMaxLinks][8]
  const float4 *rows;
  const int32_t *row_obs;
  const float4 *crows;
  int32_t n_clusters;         // clusters over all lists
  const float *q_lo, *q_hi;  // [D] composite joint limits
  // Arm pairs (i < j) whose bases are close enough for contact; other pairs
  // can never touch (every sphere stays within its arm's reach bound).
  int32_t tile_mode;       // MRPOP_TILE_*: where the tile kernel reads the rows
  int32_t n_pairs;
  const int32_t *pairs;    // [n_pairs][2]
  const uint64_t *pair_links;  // [n_pairs] bit a * 8 + b: links a, b can touch
};

constexpr int kMaxWavesPerBlock = 16;

struct DeviceBuffer {
  void *ptr = nullptr;
  size_t bytes = 0;
};

}  // namespace mrpop

struct mrpop_ctx {
  int device = 0;
  std::string last_error;
  // Scratch reused across calls (grown on demand): slot 0 edge validation,
  // 1 the planner's one-scene validations, 2 and 3 its many-scene segment
  // tables and scratch.
  mrpop::DeviceBuffer scratch[8];
  // Profiling of the validation tile kernel: event pairs recorded on the
  // launch stream, and device totals (states checked, edge states).
  bool profiling = false;
  int prof_stride = 1;       // time every prof_stride-th tile launch
  int64_t prof_seen = 0;     // tile launches since profiling was enabled
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;
  size_t ev_used = 0;
  double prof_ms = 0.0;
  int64_t prof_launches = 0; // timed launches drained so far
  uint64_t *prof_totals = nullptr;  // device [10]
  int32_t last_grid = 0, last_block = 0;  // last tile-kernel launch
  // One-launch small validations: the device arrival counter (zero between
  // launches) followed by their flag words, and the source of each launch's
  // hit token.
  uint32_t *small_arrived = nullptr;
  uint32_t small_tokens = 0;
  // Blocks that finished plans returned (device arenas, pinned host blocks),
  // kept for the next plans so that a plan allocates and frees nothing.
  std::mutex pool_mu;
  std::vector<std::pair<void *, size_t>> pool_dev, pool_pin;
  size_t pool_dev_bytes = 0, pool_pin_bytes = 0;
};

namespace mrpop {
// Host copy of one arm as given to mrpop_scene_create.
struct HostRobot {
  int32_t n_joints = 0;
  std::vector<float> dh, q_lo, q_hi, base, xyzr;
  std::vector<int32_t> link;
};
}  // namespace mrpop

struct mrpop_scene {
  mrpop_ctx *ctx = nullptr;
  std::vector<mrpop::HostRobot> h_robots;
  std::vector<float> h_env_s, h_env_b;
  mrpop::SceneDev dev{};
  void *blob = nullptr;            // one device allocation holding every array
  size_t blob_bytes = 0;
  // host copies used by the planner driver
  std::vector<float> q_lo, q_hi;   // [D]
  std::vector<int32_t> nj;         // per arm
  int32_t n_robots = 0, dof = 0, total_spheres = 0;
  // one-arm sub-scenes of the roadmaps, built by the first plan that needs
  // them and kept until the scene is destroyed (a new environment makes a new
  // scene); read-only, shared by every plan on the scene
  mutable std::vector<mrpop_scene *> arm_cache;
};

namespace mrpop {

// Record an error message on the context and return the status.
mrpop_status fail(mrpop_ctx *ctx, mrpop_status st, const std::string &msg);
// Map a HIP error to E_DEVICE (or E_NOMEM) with the call site in the message.
mrpop_status hip_fail(mrpop_ctx *ctx, hipError_t e, const char *what);
// Ensure scratch slot `slot` holds at least `bytes`.
mrpop_status scratch_slot(mrpop_ctx *ctx, int slot, size_t bytes, void **out);
// A device (pinned = false) or pinned host block of at least `bytes` from the
// context's pool (a kept block up to about twice the size), else newly
// allocated; *got is its size, to be given back to pool_free.  Safe from
// several threads.  Contents are arbitrary.
hipError_t pool_alloc(mrpop_ctx *ctx, bool pinned, size_t bytes, void **out, size_t *got);
// Returns a block to the pool, which keeps at most kPoolKeepDev / kPoolKeepPin
// bytes and frees the oldest blocks beyond that.  No queued work may use it.
void pool_free(mrpop_ctx *ctx, bool pinned, void *p, size_t bytes);
constexpr size_t kPoolKeepDev = size_t(1) << 30, kPoolKeepPin = size_t(64) << 20;

// Kernel launchers (host functions defined next to their kernels).
hipError_t launch_fk_spheres(const SceneDev &sc, const float *q, int64_t n_cfg, float *out, hipStream_t s);

struct ValidateScratch {
  int32_t *n_states;     // [E]
  int64_t *offsets;      // [E + 1]
  uint32_t *flags;       // [E] bit 0: collides, bit 1: non-finite
  uint64_t *counters;    // [16]: 0 tile queue, 1 total states, 2 states checked, 3 tiles, 4 nonfinite,
                         //       5 invalid, 6 too long, 8..15 work counts (chains, links, env tests,
                         //       exact box, rr coarse, fine sphere, fine box, fine rr)
  int64_t *block_sums;   // scan partials
  uint64_t *partials;    // [kMaxGrid][kPartialSlots] per-workgroup work counts of the tile kernel
  int32_t *tile_first;   // [kTileFirstCap] edge holding each tile's first list position
};
constexpr int kPartialSlots = 10;  // states checked, 8 work counts, tiles
// Largest batch validated in one launch from the producer's state counts.
constexpr int64_t kFusedMaxEdges = 1024;
constexpr int kMaxGrid = 8192;
constexpr int64_t kTileFirstCap = 1 << 20;
size_t validate_scratch_bytes(int64_t n_edges);
ValidateScratch validate_scratch_layout(void *base, int64_t n_edges);
// ev_pair (optional): events recorded right before and after the tile
// kernel; totals (optional): device [10] accumulators (states checked, edge
// states, then the eight work counts) added by the final kernel.
hipError_t launch_validate(const SceneDev &sc, const float *qa, const float *qb, int64_t n_edges, float res,
                           const int32_t *n_states_opt, uint8_t *out_valid, const ValidateScratch &ws,
                           hipStream_t s, const std::pair<hipEvent_t, hipEvent_t> *ev_pair = nullptr,
                           uint64_t *totals = nullptr, int32_t *grid_out = nullptr,
                           int32_t *block_out = nullptr, bool may_tune = true);
// The same for 1..kFusedMaxEdges edges in one launch, from state-count codes
// the edges' producer wrote (codes, device [n_edges]; the counts of
// state_count_code): arrived is a device counter that is zero between
// launches, ws.flags flag words that hold no value equal to token (zero or
// earlier tokens), token a value with the top bit set.  Results and
// counters as launch_validate.
hipError_t launch_validate_small(const SceneDev &sc, const float *qa, const float *qb, int64_t n_edges,
                                 const int32_t *codes, uint8_t *out_valid, const ValidateScratch &ws,
                                 uint32_t *arrived, uint32_t token, hipStream_t s,
                                 const std::pair<hipEvent_t, hipEvent_t> *ev_pair = nullptr,
                                 uint64_t *totals = nullptr, int32_t *grid_out = nullptr,
                                 int32_t *block_out = nullptr);
// Take an event pair for one profiled launch (nullptr when not profiling).
const std::pair<hipEvent_t, hipEvent_t> *profile_slot(mrpop_ctx *ctx);
// Arrival counter, flag words ([kFusedMaxEdges], written only by these
// launches) and a fresh hit token for one launch_validate_small.
hipError_t small_launch_state(mrpop_ctx *ctx, uint32_t **arrived, uint32_t **flags, uint32_t *token);

// One validation request of a many-scene launch: edges [edge0, edge0 +
// n_edges) of the flat list are (qa[i], qb[i]) of scene sc; bits go to
// out[i], the request's counters (layout of ValidateScratch::counters) to
// counters[16].  tile0 (first tile) is filled on the device.
struct ValSeg {
  SceneDev sc;
  const float *qa, *qb;
  int64_t edge0, n_edges, tile0;
  float res;
  int32_t S;  // link parts per arm (tile shape of this scene)
  uint8_t *out;
  uint64_t *counters;
};

struct SegScratch {
  int32_t *n_states, *edge_seg;  // [F]
  uint32_t *flags;               // [F]
  int64_t *offsets;              // [F + 1]
  int64_t *block_sums;
  uint64_t *batch;               // [16]: 1 total tiles, 2 tile table overflow
  uint64_t *partials;            // [kMaxGrid][kPartialSlots]
  int32_t *tile_first, *tile_seg;  // [kTileFirstCap]
};
size_t seg_scratch_bytes(int64_t n_flat);
SegScratch seg_scratch_layout(void *base, int64_t n_flat);
// Link parts per arm for a scene of n_robots arms in a launch of W waves.
int seg_link_split(int n_robots, int W);
// Waves per workgroup and whether joint sines/cosines are cached, for a
// launch whose largest scene has r_max arms.
void seg_shape(int r_max, int64_t n_flat, int *W, int *cache_sc);
// The tile-shape autotuner (validate.hip): a JSON cache file (null: none)
// whose entries are loaded now and appended to as shapes are measured, and
// whether unseen launch kinds are measured; the in-memory table is cleared.
// The defaults come from MRPOP_TUNE_CACHE and MRPOP_AUTOTUNE ("0": off).
void tuner_configure(const char *cache_file, bool enable);
int tuner_entries();
// Largest many-scene batch prepared in one workgroup, and the largest batch
// counted and scanned in one workgroup: at most kSmallScanEdges edges, and
// beyond kSmallScanOne edges at most kSmallScanLoads endpoint coordinates
// (edges x dof; one workgroup reads them all, so large composite batches go
// to the many-workgroup kernels).
constexpr int kSegSmallMax = 8;
constexpr int64_t kSmallScanEdges = 16384;
constexpr int64_t kSmallScanOne = 1024;
constexpr int64_t kSmallScanLoads = 32768;
inline bool small_scan(int64_t n_edges, int dof) {
  return n_edges <= kSmallScanOne || (n_edges <= kSmallScanEdges && n_edges * dof <= kSmallScanLoads);
}
// The same for at most kSegSmallMax consecutive segments covering
// [0, n_flat) (small_scan at the largest dof), given on the host: they travel as
// kernel arguments and are stored to d_segs (room for n_segs) by the
// preparation kernel.  Three launches instead of eight and a copy.
hipError_t launch_validate_segments_small(const ValSeg *segs, int n_segs, int r_max, int64_t n_flat, ValSeg *d_segs,
                                          const SegScratch &ws, hipStream_t s,
                                          const std::pair<hipEvent_t, hipEvent_t> *ev_pair = nullptr,
                                          uint64_t *totals = nullptr, int32_t *grid_out = nullptr,
                                          int32_t *block_out = nullptr);
// d_segs: device copy of the requests (tile0 is written there).
hipError_t launch_validate_segments(ValSeg *d_segs, int n_segs, int r_max, int64_t n_flat, const SegScratch &ws,
                                    hipStream_t s, const std::pair<hipEvent_t, hipEvent_t> *ev_pair = nullptr,
                                    uint64_t *totals = nullptr, int32_t *grid_out = nullptr,
                                    int32_t *block_out = nullptr);

}  // namespace mrpop
