// C ABI entry points: contexts, scenes, argument checks and dispatch.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "mrpop_internal.h"

namespace {
thread_local std::string g_create_error;
}

namespace mrpop {

mrpop_status fail(mrpop_ctx *ctx, mrpop_status st, const std::string &msg) {
  if (ctx) ctx->last_error = msg;
  else g_create_error = msg;
  return st;
}

mrpop_status hip_fail(mrpop_ctx *ctx, hipError_t e, const char *what) {
  std::string msg = std::string(what) + ": " + hipGetErrorString(e);
  return fail(ctx, e == hipErrorOutOfMemory ? MRPOP_E_NOMEM : MRPOP_E_DEVICE, msg);
}

mrpop_status scratch_slot(mrpop_ctx *ctx, int slot, size_t bytes, void **out) {
  DeviceBuffer &b = ctx->scratch[slot];
  if (b.bytes < bytes) {
    if (b.ptr) {
      hipError_t e = hipFree(b.ptr);
      b.ptr = nullptr;
      b.bytes = 0;
      if (e != hipSuccess) return hip_fail(ctx, e, "hipFree(scratch)");
    }
    size_t want = std::max<size_t>(bytes + bytes / 4, 1 << 16);
    hipError_t e = hipMalloc(&b.ptr, want);
    if (e != hipSuccess) {
      b.ptr = nullptr;
      return hip_fail(ctx, e, "hipMalloc(scratch)");
    }
    b.bytes = want;
  }
  *out = b.ptr;
  return MRPOP_OK;
}

hipError_t pool_alloc(mrpop_ctx *ctx, bool pinned, size_t bytes, void **out, size_t *got) {
  bytes = std::max<size_t>(bytes, 256);
  {
    std::lock_guard<std::mutex> lk(ctx->pool_mu);
    auto &v = pinned ? ctx->pool_pin : ctx->pool_dev;
    size_t best = v.size();
    for (size_t i = 0; i < v.size(); ++i)
      if (v[i].second >= bytes && v[i].second <= 2 * bytes + (size_t(1) << 20) &&
          (best == v.size() || v[i].second < v[best].second))
        best = i;
    if (best < v.size()) {
      *out = v[best].first;
      *got = v[best].second;
      (pinned ? ctx->pool_pin_bytes : ctx->pool_dev_bytes) -= v[best].second;
      v.erase(v.begin() + (std::ptrdiff_t)best);
      return hipSuccess;
    }
  }
  *got = bytes;
  return pinned ? hipHostMalloc(out, bytes) : hipMalloc(out, bytes);
}

void pool_free(mrpop_ctx *ctx, bool pinned, void *p, size_t bytes) {
  if (!p) return;
  std::vector<std::pair<void *, size_t>> drop;
  {
    std::lock_guard<std::mutex> lk(ctx->pool_mu);
    auto &v = pinned ? ctx->pool_pin : ctx->pool_dev;
    size_t &total = pinned ? ctx->pool_pin_bytes : ctx->pool_dev_bytes;
    v.push_back({p, bytes});
    total += bytes;
    const size_t keep = pinned ? kPoolKeepPin : kPoolKeepDev;
    while (total > keep && !v.empty()) {
      drop.push_back(v.front());
      total -= v.front().second;
      v.erase(v.begin());
    }
  }
  for (auto &b : drop) (void)(pinned ? hipHostFree(b.first) : hipFree(b.first));
}

const std::pair<hipEvent_t, hipEvent_t> *profile_slot(mrpop_ctx *ctx) {
  if (!ctx->profiling) return nullptr;
  if (ctx->prof_seen++ % ctx->prof_stride != 0) return nullptr;  // counted, not timed
  if (ctx->ev_used == ctx->ev_pool.size()) {
    std::pair<hipEvent_t, hipEvent_t> p{nullptr, nullptr};
    // timing-only events: no system-scope fence when they complete (no cache
    // write-back and invalidation that would lengthen what they time).  An
    // event-timed launch then costs about 13 us of dispatch instead of 14-24
    // with a device-scope release (a plain launch: about 5 us).
    if (hipEventCreateWithFlags(&p.first, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    if (hipEventCreateWithFlags(&p.second, hipEventDisableSystemFence) != hipSuccess) {
      hipEventDestroy(p.first);
      return nullptr;
    }
    ctx->ev_pool.push_back(p);
  }
  return &ctx->ev_pool[ctx->ev_used++];
}

hipError_t small_launch_state(mrpop_ctx *ctx, uint32_t **arrived, uint32_t **flags, uint32_t *token) {
  // one allocation: the arrival counter, then kFusedMaxEdges flag words that
  // only these launches write (zero, or an earlier launch's token)
  if (!ctx->small_arrived) {
    const size_t bytes = 256 + sizeof(uint32_t) * kFusedMaxEdges;
    hipError_t e = hipMalloc((void **)&ctx->small_arrived, bytes);
    if (e != hipSuccess) {
      ctx->small_arrived = nullptr;
      return e;
    }
    e = hipMemset(ctx->small_arrived, 0, bytes);
    if (e != hipSuccess) return e;
  }
  *flags = ctx->small_arrived + 64;
  // tokens 0x80000001, 0x80000002, ...: the top bit keeps them apart from
  // the general path's flag values; when the sequence wraps, the words are
  // cleared so that no word keeps a token about to be reused
  ctx->small_tokens = (ctx->small_tokens + 1u) & 0x7fffffffu;
  if (ctx->small_tokens == 0u) {
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemset(*flags, 0, sizeof(uint32_t) * kFusedMaxEdges);
    if (e != hipSuccess) return e;
    ctx->small_tokens = 1u;
  }
  *arrived = ctx->small_arrived;
  *token = 0x80000000u | ctx->small_tokens;
  return hipSuccess;
}

}  // namespace mrpop

// ---------------------------------------------------------------------------
// Fixed device scratch of mrpop_validate_edges_noalloc
// ---------------------------------------------------------------------------

namespace {

constexpr size_t kNoAllocScratchBytes = size_t(6) << 20;
constexpr int kNoAllocMaxDevices = 64;

// Every GPU the library runs on holds its own copy of this array until the
// process ends.  In host code its name is only a stand-in: the kernels get the
// device address that hipGetSymbolAddress returns for the current device,
// taken once per device when the first context on it is created.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_noalloc_mu;
void *g_noalloc_ptr[kNoAllocMaxDevices] = {};

// With `device` current: the device address of `scratch` on it (once).
hipError_t noalloc_scratch_init(int device) {
  if (device < 0 || device >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (g_noalloc_ptr[device]) return hipSuccess;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_noalloc_ptr[device] = p;
  return hipSuccess;
}

void *noalloc_scratch_ptr(int device) {
  if (device < 0 || device >= kNoAllocMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  return g_noalloc_ptr[device];
}

}  // namespace

using namespace mrpop;

extern "C" {

const char *mrpop_version(void) { return "mrpop-mi355x 0.1 (gfx950)"; }

mrpop_status mrpop_ctx_create(int device, mrpop_ctx **out) {
  if (!out) return fail(nullptr, MRPOP_E_INVALID_ARG, "ctx_create: out is NULL");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDeviceCount");
  if (device < 0 || device >= n) return fail(nullptr, MRPOP_E_INVALID_ARG, "ctx_create: no such device");
  e = hipSetDevice(device);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipSetDevice");
  e = noalloc_scratch_init(device);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetSymbolAddress(scratch)");
  mrpop_ctx *c = new mrpop_ctx();
  c->device = device;
  *out = c;
  return MRPOP_OK;
}

void mrpop_ctx_destroy(mrpop_ctx *ctx) {
  if (!ctx) return;
  hipSetDevice(ctx->device);
  for (auto &b : ctx->scratch)
    if (b.ptr) hipFree(b.ptr);
  for (auto &p : ctx->ev_pool) {
    hipEventDestroy(p.first);
    hipEventDestroy(p.second);
  }
  if (ctx->prof_totals) hipFree(ctx->prof_totals);
  if (ctx->small_arrived) hipFree(ctx->small_arrived);
  for (auto &b : ctx->pool_dev) hipFree(b.first);
  for (auto &b : ctx->pool_pin) hipHostFree(b.first);
  delete ctx;
}

mrpop_status mrpop_profile_enable(mrpop_ctx *ctx, int enable) {
  if (!ctx) return fail(nullptr, MRPOP_E_INVALID_ARG, "profile_enable: ctx is NULL");
  if (enable < 0) return fail(ctx, MRPOP_E_INVALID_ARG, "profile_enable: negative stride");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  ctx->profiling = enable != 0;
  ctx->prof_stride = enable > 1 ? enable : 1;
  ctx->prof_seen = 0;
  ctx->ev_used = 0;
  ctx->prof_ms = 0.0;
  ctx->prof_launches = 0;
  if (enable) {
    if (!ctx->prof_totals) {
      e = hipMalloc((void **)&ctx->prof_totals, 10 * sizeof(uint64_t));
      if (e != hipSuccess) {
        ctx->prof_totals = nullptr;
        ctx->profiling = false;
        return hip_fail(ctx, e, "hipMalloc(profile)");
      }
    }
    e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemset(ctx->prof_totals, 0, 10 * sizeof(uint64_t));
    if (e != hipSuccess) return hip_fail(ctx, e, "profile_enable");
  }
  return MRPOP_OK;
}

// Sum the elapsed time of the recorded event pairs and recycle them.
static mrpop_status drain_events(mrpop_ctx *ctx) {
  for (size_t i = 0; i < ctx->ev_used; ++i) {
    hipError_t e = hipEventSynchronize(ctx->ev_pool[i].second);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ctx->ev_pool[i].first, ctx->ev_pool[i].second);
    if (e != hipSuccess) return hip_fail(ctx, e, "profile events");
    ctx->prof_ms += ms;
    ctx->prof_launches++;
  }
  ctx->ev_used = 0;
  return MRPOP_OK;
}

mrpop_status mrpop_profile_read(mrpop_ctx *ctx, mrpop_kernel_profile *out) {
  if (!ctx) return fail(nullptr, MRPOP_E_INVALID_ARG, "profile_read: ctx is NULL");
  if (!out) return fail(ctx, MRPOP_E_INVALID_ARG, "profile_read: out is NULL");
  std::memset(out, 0, sizeof(*out));
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  mrpop_status st = drain_events(ctx);
  if (st != MRPOP_OK) return st;
  out->launches = ctx->prof_seen;
  out->timed_launches = ctx->prof_launches;
  out->kernel_ms = ctx->prof_ms;
  out->grid_blocks = ctx->last_grid;
  out->block_threads = ctx->last_block;
  if (ctx->prof_totals) {
    uint64_t t[10];
    e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(t, ctx->prof_totals, sizeof(t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(ctx, e, "profile_read");
    out->states_checked = (int64_t)t[0];
    out->edge_states = (int64_t)t[1];
    for (int i = 0; i < 8; ++i) out->work[i] = (int64_t)t[2 + i];
  }
  return MRPOP_OK;
}

const char *mrpop_last_error(const mrpop_ctx *ctx) {
  return ctx ? ctx->last_error.c_str() : g_create_error.c_str();
}

// ---------------------------------------------------------------------------
// Scene packing
// ---------------------------------------------------------------------------

static bool finite_all(const float *p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

static bool same_model(const mrpop_robot &a, const mrpop_robot &b) {
  if (a.n_joints != b.n_joints || a.n_spheres != b.n_spheres) return false;
  if (std::memcmp(a.dh, b.dh, sizeof(float) * 4 * a.n_joints)) return false;
  if (std::memcmp(a.sphere_link, b.sphere_link, sizeof(int32_t) * a.n_spheres)) return false;
  if (std::memcmp(a.sphere_xyzr, b.sphere_xyzr, sizeof(float) * 4 * a.n_spheres)) return false;
  return true;
}

// Round a non-negative double up to the next float that is >= it.
static float round_up_f(double v) {
  float f = (float)v;
  if ((double)f < v) f = std::nextafter(f, INFINITY);
  return f;
}

// Inflation of the per-link bounding sphere.  The coarse level is a filter
// only: a fine sphere that touches an obstacle lies inside its link's coarse
// sphere with this much room to spare, so single-precision rounding in the
// coarse test can never hide a contact.
static constexpr double kCoarseInflate = 1e-4;

// Two-level coarse filter: a link's obstacle list of at least
// kClusterMinObstacles entries may group every kClusterSize consecutive rows
// into a cluster with a bounding sphere of its own, tested first.  Where
// obstacles are sparse the clusters are large and nearly all pass, so the
// extra level only adds tests; a list keeps them only when an estimate of
// the tests per link says they pay.
static constexpr int kClusterMinObstacles = 64;
// Clusters are kept when the estimated tests are at most this fraction of
// the tests without them (the estimate is per lane; a wave tests a
// cluster's members when any of its lanes passes, which costs more).
static constexpr double kClusterGain = 0.5;
// Slack of the reach test that builds the per-link obstacle lists, in metres
// (covers single-precision rounding of the chain, far below it).
static constexpr double kReachMargin = 1e-3;

// Order of the points along a Morton (Z-order) curve over their bounding
// box, ten bits per axis (ties keep the input order).
static std::vector<int> morton_order(const std::vector<float4> &pts, int n) {
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int i = 0; i < n; ++i) {
    const double v[3] = {pts[i].x, pts[i].y, pts[i].z};
    for (int a = 0; a < 3; ++a) { lo[a] = std::min(lo[a], v[a]); hi[a] = std::max(hi[a], v[a]); }
  }
  auto spread = [](uint64_t x) {  // the ten bits of x to every third bit
    x &= 0x3ff;
    x = (x | (x << 16)) & 0x30000ff;
    x = (x | (x << 8)) & 0x300f00f;
    x = (x | (x << 4)) & 0x30c30c3;
    x = (x | (x << 2)) & 0x9249249;
    return x;
  };
  std::vector<uint64_t> code(n);
  for (int i = 0; i < n; ++i) {
    const double v[3] = {pts[i].x, pts[i].y, pts[i].z};
    uint64_t c = 0;
    for (int a = 0; a < 3; ++a) {
      const double span = hi[a] - lo[a];
      const uint64_t q = span > 0 ? (uint64_t)std::min(1023.0, std::floor((v[a] - lo[a]) / span * 1023.0)) : 0;
      c |= spread(q) << a;
    }
    code[i] = c;
  }
  std::vector<int> ord(n);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return code[a] < code[b]; });
  return ord;
}

// Link centres of every arm at seeded random configurations within the
// joint limits, for the cluster estimate: [R][kMaxLinks][samples] x, y, z
// (recentred world frame; forward kinematics on the host in double
// precision, with the kernels' convention; links without spheres left 0).
static std::vector<double> sample_link_centres(const mrpop_robot *robots, int n_robots,
                                               const std::vector<int32_t> &model_of, const std::vector<float4> &dh,
                                               const std::vector<float> &th, const std::vector<float4> &coarse,
                                               const std::vector<float> &base, int samples) {
  std::vector<double> out((size_t)n_robots * kMaxLinks * samples * 3, 0.0);
  uint64_t sm = 0x2545f4914f6cdd1dull;
  auto next_u01 = [&sm]() {  // splitmix64 (Steele, Lea and Flood, 2014), top 53 bits
    uint64_t z = (sm += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return (double)((z ^ (z >> 31)) >> 11) * 0x1.0p-53;
  };
  for (int r = 0; r < n_robots; ++r) {
    const mrpop_robot &rb = robots[r];
    const int m = model_of[r];
    for (int k = 0; k < samples; ++k) {
      double F[12];
      for (int i = 0; i < 12; ++i) F[i] = base[(size_t)r * 12 + i];
      for (int l = 0; l <= rb.n_joints; ++l) {
        if (l > 0) {
          // F <- F RotX(alpha) TransX(a) RotZ(theta) TransZ(d), row by row
          const float4 p = dh[(size_t)m * kMaxJoints + l - 1];
          const double q = rb.q_lo[l - 1] + next_u01() * ((double)rb.q_hi[l - 1] - rb.q_lo[l - 1]) +
                           th[(size_t)m * kMaxJoints + l - 1];
          const double c = std::cos(q), sn = std::sin(q);
          for (int row = 0; row < 3; ++row) {
            double *R = F + 4 * row;
            const double u = R[1] * p.z + R[2] * p.w, n2 = R[2] * p.z - R[1] * p.w;
            R[3] += R[0] * p.x + n2 * p.y;
            const double n0 = R[0] * c + u * sn, n1 = u * c - R[0] * sn;
            R[0] = n0;
            R[1] = n1;
            R[2] = n2;
          }
        }
        const float4 cv = coarse[(size_t)m * kMaxLinks + l];
        if (cv.w < 0) continue;
        double *o = &out[(((size_t)r * kMaxLinks + l) * samples + k) * 3];
        o[0] = F[0] * cv.x + F[1] * cv.y + F[2] * cv.z + F[3];
        o[1] = F[4] * cv.x + F[5] * cv.y + F[6] * cv.z + F[7];
        o[2] = F[8] * cv.x + F[9] * cv.y + F[10] * cv.z + F[11];
      }
    }
  }
  return out;
}

struct Blob {
  std::vector<unsigned char> host;
  size_t add(const void *p, size_t bytes) {
    size_t off = (host.size() + 255) & ~size_t(255);
    host.resize(off + bytes);
    if (bytes) std::memcpy(host.data() + off, p, bytes);
    return off;
  }
};

mrpop_status mrpop_scene_create(mrpop_ctx *ctx, const mrpop_robot *robots, int32_t n_robots,
                                const mrpop_env *env, mrpop_scene **out) {
  if (!ctx) return fail(nullptr, MRPOP_E_INVALID_ARG, "scene_create: ctx is NULL");
  if (!out || !robots || !env) return fail(ctx, MRPOP_E_INVALID_ARG, "scene_create: NULL argument");
  *out = nullptr;
  if (n_robots < 1 || n_robots > MRPOP_MAX_ROBOTS)
    return fail(ctx, MRPOP_E_INVALID_ARG, "scene_create: n_robots out of range");
  for (int r = 0; r < n_robots; ++r) {
    const mrpop_robot &rb = robots[r];
    if (rb.n_joints < 1 || rb.n_joints > MRPOP_MAX_JOINTS)
      return fail(ctx, MRPOP_E_INVALID_ARG, "scene_create: n_joints out of range");
    if (rb.n_spheres < 1 || rb.n_spheres > MRPOP_MAX_SPHERES)
      return fail(ctx, MRPOP_E_INVALID_ARG, "scene_create: n_spheres out of range");
    if (!rb.dh || !rb.q_lo || !rb.q_hi || !rb.base_tf || !rb.sphere_link || !rb.sphere_xyzr)
      return fail(ctx, MRPOP_E_INVALID_ARG, "scene_create: NULL robot array");
    if (!finite_all(rb.dh, 4 * rb.n_joints) || !finite_all(rb.q_lo, rb.n_joints) ||
        !finite_all(rb.q_hi, rb.n_joints) || !finite_all(rb.base_tf, 12) ||
        !finite_all(rb.sphere_xyzr, 4 * rb.n_spheres))
      return fail(ctx, MRPOP_E_NONFINITE, "scene_create: non-finite robot data");
    for (int j = 0; j < rb.n_joints; ++j)
      if (rb.q_lo[j] > rb.q_hi[j]) return fail(ctx, MRPOP_E_INVALID_ARG, "scene_create: q_lo > q_hi");
    for (int i = 0; i < rb.n_spheres; ++i) {
      if (rb.sphere_link[i] < 0 || rb.sphere_link[i] > rb.n_joints)
        return fail(ctx, MRPOP_E_INVALID_ARG, "scene_create: sphere_link out of range");
      if (rb.sphere_xyzr[4 * i + 3] < 0) return fail(ctx, MRPOP_E_INVALID_ARG, "scene_create: negative radius");
    }
  }
  if (env->n_spheres < 0 || env->n_spheres > MRPOP_MAX_ENV || env->n_boxes < 0 || env->n_boxes > MRPOP_MAX_ENV)
    return fail(ctx, MRPOP_E_INVALID_ARG, "scene_create: obstacle count out of range");
  if ((env->n_spheres && !env->spheres) || (env->n_boxes && !env->boxes))
    return fail(ctx, MRPOP_E_INVALID_ARG, "scene_create: NULL obstacle array");
  if (!finite_all(env->spheres, 4 * (size_t)env->n_spheres) || !finite_all(env->boxes, 6 * (size_t)env->n_boxes))
    return fail(ctx, MRPOP_E_NONFINITE, "scene_create: non-finite obstacle");
  for (int k = 0; k < env->n_spheres; ++k)
    if (env->spheres[4 * k + 3] < 0) return fail(ctx, MRPOP_E_INVALID_ARG, "scene_create: negative radius");
  for (int k = 0; k < env->n_boxes; ++k)
    for (int a = 0; a < 3; ++a)
      if (env->boxes[6 * k + a] > env->boxes[6 * k + 3 + a])
        return fail(ctx, MRPOP_E_INVALID_ARG, "scene_create: box lo > hi");

  // Models: one shared model when every arm is identical.
  bool homog = true;
  for (int r = 1; r < n_robots; ++r) homog = homog && same_model(robots[0], robots[r]);
  std::vector<int32_t> model_of(n_robots);
  std::vector<const mrpop_robot *> models;
  for (int r = 0; r < n_robots; ++r) {
    if (homog && r > 0) { model_of[r] = 0; continue; }
    model_of[r] = (int32_t)models.size();
    models.push_back(&robots[r]);
  }
  const int M = (int)models.size();
  int sph_stride = 0;
  for (auto *m : models) sph_stride = std::max(sph_stride, m->n_spheres);

  // Recentre the world on the middle of the bases' bounding box so that
  // single-precision coordinates stay small.
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int r = 0; r < n_robots; ++r)
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], (double)robots[r].base_tf[4 * a + 3]);
      hi[a] = std::max(hi[a], (double)robots[r].base_tf[4 * a + 3]);
    }
  double org[3];
  for (int a = 0; a < 3; ++a) org[a] = (double)(float)(0.5 * (lo[a] + hi[a]));

  std::vector<int32_t> nj(M), link_start((size_t)M * (kMaxLinks + 1), 0), fine_src((size_t)M * sph_stride, 0);
  std::vector<float4> dh((size_t)M * kMaxJoints, float4{0, 0, 1, 0}), fine((size_t)M * sph_stride, float4{0, 0, 0, 0}),
      coarse((size_t)M * kMaxLinks, float4{0, 0, 0, -1});
  std::vector<float> th((size_t)M * kMaxJoints, 0.f);
  for (int m = 0; m < M; ++m) {
    const mrpop_robot &rb = *models[m];
    nj[m] = rb.n_joints;
    for (int j = 0; j < rb.n_joints; ++j) {
      double alpha = rb.dh[4 * j + 2];
      dh[(size_t)m * kMaxJoints + j] = float4{rb.dh[4 * j], rb.dh[4 * j + 1], (float)std::cos(alpha), (float)std::sin(alpha)};
      th[(size_t)m * kMaxJoints + j] = rb.dh[4 * j + 3];
    }
    // group spheres by link (stable)
    std::vector<int> order(rb.n_spheres);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return rb.sphere_link[a] < rb.sphere_link[b]; });
    int32_t *ls = &link_start[(size_t)m * (kMaxLinks + 1)];
    for (int i = 0; i < rb.n_spheres; ++i) {
      int src = order[i];
      fine[(size_t)m * sph_stride + i] = float4{rb.sphere_xyzr[4 * src], rb.sphere_xyzr[4 * src + 1],
                                                rb.sphere_xyzr[4 * src + 2], rb.sphere_xyzr[4 * src + 3]};
      fine_src[(size_t)m * sph_stride + i] = src;
      ls[rb.sphere_link[src] + 1]++;
    }
    for (int l = 0; l < kMaxLinks; ++l) ls[l + 1] += ls[l];
    // coarse sphere per link: middle of the bounding box of the link's sphere
    // centres, radius reaching past every fine sphere, plus the inflation
    for (int l = 0; l <= rb.n_joints; ++l) {
      if (ls[l + 1] == ls[l]) continue;
      double bl[3] = {INFINITY, INFINITY, INFINITY}, bh[3] = {-INFINITY, -INFINITY, -INFINITY};
      for (int i = ls[l]; i < ls[l + 1]; ++i) {
        const float4 f = fine[(size_t)m * sph_stride + i];
        const double p[3] = {f.x, f.y, f.z};
        for (int a = 0; a < 3; ++a) { bl[a] = std::min(bl[a], p[a]); bh[a] = std::max(bh[a], p[a]); }
      }
      float c[3];
      for (int a = 0; a < 3; ++a) c[a] = (float)(0.5 * (bl[a] + bh[a]));
      double rad = 0;
      for (int i = ls[l]; i < ls[l + 1]; ++i) {
        const float4 f = fine[(size_t)m * sph_stride + i];
        double dx = (double)f.x - c[0], dy = (double)f.y - c[1], dz = (double)f.z - c[2];
        rad = std::max(rad, std::sqrt(dx * dx + dy * dy + dz * dz) + (double)f.w);
      }
      coarse[(size_t)m * kMaxLinks + l] = float4{c[0], c[1], c[2], round_up_f(rad + kCoarseInflate)};
    }
  }
  std::vector<int32_t> q_off(n_robots), s_out(n_robots);
  std::vector<float> base((size_t)n_robots * 12);
  int dof = 0, S = 0;
  for (int r = 0; r < n_robots; ++r) {
    q_off[r] = dof;
    s_out[r] = S;
    dof += robots[r].n_joints;
    S += robots[r].n_spheres;
    for (int i = 0; i < 12; ++i) base[(size_t)r * 12 + i] = robots[r].base_tf[i];
    for (int a = 0; a < 3; ++a) base[(size_t)r * 12 + 4 * a + 3] = (float)((double)robots[r].base_tf[4 * a + 3] - org[a]);
  }
  std::vector<float4> env_s(std::max(1, env->n_spheres)), env_b(2 * (size_t)std::max(1, env->n_boxes));
  for (int k = 0; k < env->n_spheres; ++k)
    env_s[k] = float4{(float)((double)env->spheres[4 * k] - org[0]), (float)((double)env->spheres[4 * k + 1] - org[1]),
                      (float)((double)env->spheres[4 * k + 2] - org[2]), env->spheres[4 * k + 3]};
  for (int k = 0; k < env->n_boxes; ++k) {
    const float *b = env->boxes + 6 * k;
    env_b[2 * k] = float4{(float)((double)b[0] - org[0]), (float)((double)b[1] - org[1]), (float)((double)b[2] - org[2]), 0.f};
    env_b[2 * k + 1] = float4{(float)((double)b[3] - org[0]), (float)((double)b[4] - org[1]), (float)((double)b[5] - org[2]), 0.f};
  }
  // Expanded-form coarse filter tables (see SceneDev).  delta covers the
  // rounding error of the single-precision expanded test: near a contact every
  // point involved lies within M of the origin, the table entry is rounded
  // once (|B| <= 2 M^2), the three FMAs round partial sums of size <= 4 M^2
  // and -|c|^2 takes three roundings of size <= M^2, so the computed value of
  // d^2 - R^2 is off by at most eps = 20 u M^2 (u = 2^-24).  Testing against
  // R' = sqrt(R^2 + eps) keeps every true contact, and R' - R is at most
  // min(sqrt(eps), eps / (2 R)).
  double reach = 0.0;
  for (int m = 0; m < M; ++m) {
    const mrpop_robot &rb = *models[m];
    double chain = 0.0, far = 0.0;
    for (int j = 0; j < rb.n_joints; ++j) chain += std::hypot((double)rb.dh[4 * j], (double)rb.dh[4 * j + 1]);
    for (int i = 0; i < rb.n_spheres; ++i)
      far = std::max(far, std::hypot(std::hypot((double)rb.sphere_xyzr[4 * i], (double)rb.sphere_xyzr[4 * i + 1]),
                                     (double)rb.sphere_xyzr[4 * i + 2]) + (double)rb.sphere_xyzr[4 * i + 3]);
    reach = std::max(reach, chain + far);
  }
  double base_far = 0.0, obs_r = 0.0, rc_min = INFINITY;
  for (int r = 0; r < n_robots; ++r)
    base_far = std::max(base_far, std::hypot(std::hypot((double)base[(size_t)r * 12 + 3], (double)base[(size_t)r * 12 + 7]),
                                             (double)base[(size_t)r * 12 + 11]));
  std::vector<double> box_rad(std::max(1, env->n_boxes));
  for (int k = 0; k < env->n_spheres; ++k) obs_r = std::max(obs_r, (double)env->spheres[4 * k + 3]);
  for (int k = 0; k < env->n_boxes; ++k) {
    const float *b = env->boxes + 6 * k;
    box_rad[k] = 0.5 * std::sqrt((double)(b[3] - b[0]) * (b[3] - b[0]) + (double)(b[4] - b[1]) * (b[4] - b[1]) +
                                 (double)(b[5] - b[2]) * (b[5] - b[2]));
    obs_r = std::max(obs_r, box_rad[k]);
  }
  double rc_max = 0.0;
  for (const float4 &cv : coarse)
    if (cv.w >= 0) { rc_min = std::min(rc_min, (double)cv.w); rc_max = std::max(rc_max, (double)cv.w); }
  auto delta_for = [&](double obstacle_r) {  // delta for bounding radii up to obstacle_r
    const double Mx = base_far + reach + rc_max + obstacle_r;
    const double eps = 20.0 * std::ldexp(1.0, -24) * Mx * Mx;
    return std::max(1e-4, std::min(std::sqrt(eps), eps / (2.0 * std::max(rc_min, 1e-30))));
  };
  const double delta = delta_for(obs_r);
  // bounding sphere of every obstacle (spheres, then boxes): centre (single
  // precision) and radius
  const int NS = env->n_spheres, NB = env->n_boxes, NO = NS + NB;
  std::vector<float4> bound(std::max(1, NO));
  std::vector<double> bound_r(std::max(1, NO));
  {
    for (int k = 0; k < NS; ++k) {
      bound[k] = env_s[k];
      bound_r[k] = (double)env_s[k].w;
    }
    for (int k = 0; k < NB; ++k) {
      const float4 lo = env_b[2 * k], hi = env_b[2 * k + 1];
      const float mx = 0.5f * (lo.x + hi.x), my = 0.5f * (lo.y + hi.y), mz = 0.5f * (lo.z + hi.z);
      // radius from the rounded centre to the farthest corner
      double far = 0.0;
      for (int cx = 0; cx < 2; ++cx)
        for (int cy = 0; cy < 2; ++cy)
          for (int cz = 0; cz < 2; ++cz) {
            const double dx = (double)(cx ? hi.x : lo.x) - mx, dy = (double)(cy ? hi.y : lo.y) - my,
                         dz = (double)(cz ? hi.z : lo.z) - mz;
            far = std::max(far, std::sqrt(dx * dx + dy * dy + dz * dz));
          }
      bound[NS + k] = float4{mx, my, mz, 0.f};
      bound_r[NS + k] = far;
    }
  }

  // Reach of every link: its coarse sphere stays within reach(l) =
  // sum_{j <= l} |(a_{j-1}, d_j)| + |c_l| + r_l of its arm's base origin in
  // every configuration (a joint step moves the frame's origin by
  // (a, -d sin alpha, d cos alpha), of length |(a, d)|; c_l is the coarse
  // centre in the link's frame).
  std::vector<double> link_reach((size_t)M * kMaxLinks, -1.0);
  for (int m = 0; m < M; ++m) {
    const mrpop_robot &rb = *models[m];
    double chain = 0.0;
    for (int l = 0; l <= rb.n_joints && l < kMaxLinks; ++l) {
      if (l > 0) chain += std::hypot((double)rb.dh[4 * (l - 1)], (double)rb.dh[4 * (l - 1) + 1]);
      const float4 cv = coarse[(size_t)m * kMaxLinks + l];
      if (cv.w < 0) continue;
      link_reach[(size_t)m * kMaxLinks + l] =
          chain + std::sqrt((double)cv.x * cv.x + (double)cv.y * cv.y + (double)cv.z * cv.z) + (double)cv.w + 1e-3;
    }
  }

  // Per-(arm, link) obstacle lists.  Link l of arm r can touch obstacle k
  // only if k's bounding sphere comes within reach(l) of the arm's base
  // origin, so each list keeps just those obstacles, in Morton order of their
  // bounding centres (10 bits per axis over the obstacles' bounding box).
  // Each list's rows are padded to a multiple of eight with never-passing
  // rows, and row_obs names each row's obstacle.  A list of at least
  // kClusterMinObstacles obstacles may also get clusters: every eight
  // consecutive rows form one, whose sphere (centre the mean of the
  // members' bounding centres, radius reaching past every member's bounding
  // sphere) contains every member, so a link that touches a member passes
  // the cluster's test.  Cluster rows take the same expanded form, with
  // delta recomputed for the larger radii.  A list keeps its clusters only
  // when the estimated tests per link with them (one per cluster plus eight
  // per cluster that passes, over the link's centres at seeded random
  // configurations) are at most kClusterGain of its length.
  std::vector<int> order(NO);
  std::iota(order.begin(), order.end(), 0);
  if (NO > 1) order = morton_order(bound, NO);
  const int n_samples = 128;
  std::vector<double> centres;
  bool sampled = false;
  std::vector<int32_t> lists((size_t)n_robots * kMaxLinks * 8, 0);
  std::vector<float4> rows, crows;
  std::vector<int32_t> row_obs;
  const float4 never{0.f, 0.f, 0.f, 3.0e38f};
  int64_t NC = 0;
  std::vector<int> L;
  for (int r = 0; r < n_robots; ++r) {
    const int m = model_of[r];
    const double bx = base[(size_t)r * 12 + 3], by = base[(size_t)r * 12 + 7], bz = base[(size_t)r * 12 + 11];
    for (int l = 0; l < kMaxLinks; ++l) {
      int32_t *meta = &lists[((size_t)r * kMaxLinks + l) * 8];
      meta[0] = (int32_t)rows.size();
      meta[3] = (int32_t)crows.size();
      const float4 cv = coarse[(size_t)m * kMaxLinks + l];
      if (cv.w < 0 || l > models[m]->n_joints) continue;
      const double reach_l = link_reach[(size_t)m * kMaxLinks + l];
      L.clear();
      for (int k : order) {
        const double dx = (double)bound[k].x - bx, dy = (double)bound[k].y - by, dz = (double)bound[k].z - bz;
        if (std::sqrt(dx * dx + dy * dy + dz * dz) <= reach_l + bound_r[k] + kReachMargin) L.push_back(k);
      }
      const int n = (int)L.size(), n8 = (n + 7) & ~7;
      for (int k : L) {
        const float4 o = bound[k];
        const double o2 = (double)o.x * o.x + (double)o.y * o.y + (double)o.z * o.z;
        const double R = (double)cv.w + bound_r[k] + delta;
        rows.push_back(float4{-2.f * o.x, -2.f * o.y, -2.f * o.z, (float)(o2 - R * R)});
        row_obs.push_back(k);
      }
      rows.resize((size_t)meta[0] + n8, never);
      row_obs.resize((size_t)meta[0] + n8, 0);
      meta[1] = n8;
      meta[2] = n;
      if (n < kClusterMinObstacles) continue;
      const int nc = (n + kClusterSize - 1) / kClusterSize;
      std::vector<float4> cc(nc);
      std::vector<double> cr(nc, 0.0);
      double cr_max = 0.0;
      for (int c = 0; c < nc; ++c) {
        const int i0 = c * kClusterSize, i1 = std::min(n, i0 + kClusterSize);
        double sx = 0, sy = 0, sz = 0;
        for (int i = i0; i < i1; ++i) { sx += bound[L[i]].x; sy += bound[L[i]].y; sz += bound[L[i]].z; }
        cc[c] = float4{(float)(sx / (i1 - i0)), (float)(sy / (i1 - i0)), (float)(sz / (i1 - i0)), 0.f};
        for (int i = i0; i < i1; ++i) {
          const float4 o = bound[L[i]];
          const double dx = (double)o.x - cc[c].x, dy = (double)o.y - cc[c].y, dz = (double)o.z - cc[c].z;
          cr[c] = std::max(cr[c], std::sqrt(dx * dx + dy * dy + dz * dz) + bound_r[L[i]]);
        }
        cr_max = std::max(cr_max, cr[c]);
      }
      const double delta_c = delta_for(std::max(obs_r, cr_max));
      if (!sampled) {
        centres = sample_link_centres(robots, n_robots, model_of, dh, th, coarse, base, n_samples);
        sampled = true;
      }
      const int S = std::max(8, std::min(n_samples, 250000 / nc));
      double tests = 0.0;
      for (int k = 0; k < S; ++k) {
        const double *x = &centres[(((size_t)r * kMaxLinks + l) * n_samples + k) * 3];
        tests += nc;
        for (int c = 0; c < nc; ++c) {
          const double dx = x[0] - cc[c].x, dy = x[1] - cc[c].y, dz = x[2] - cc[c].z;
          const double R = (double)cv.w + cr[c] + delta_c;
          if (dx * dx + dy * dy + dz * dz < R * R) tests += kClusterSize;
        }
      }
      if (tests / S > kClusterGain * n) continue;
      for (int c = 0; c < nc; ++c) {
        const float4 o = cc[c];
        const double o2 = (double)o.x * o.x + (double)o.y * o.y + (double)o.z * o.z;
        const double R = (double)cv.w + cr[c] + delta_c;
        crows.push_back(float4{-2.f * o.x, -2.f * o.y, -2.f * o.z, (float)(o2 - R * R)});
      }
      crows.resize((size_t)meta[3] + ((nc + 7) & ~7), never);
      meta[4] = (nc + 7) & ~7;
      meta[5] = nc;
      NC += nc;
    }
  }
  // one group of padding past the last list (the prefetch of the next group)
  rows.resize(rows.size() + 4, never);
  row_obs.resize(row_obs.size() + 4, 0);
  crows.resize(crows.size() + 4, never);

  // Arm pairs and, per pair, the link pairs that can touch: links a, b of
  // arms i, j never meet when the bases are farther apart than reach_i(a) +
  // reach_j(b).  Bit a * 8 + b of a pair's mask marks a possible link pair.
  std::vector<int32_t> pairs;
  std::vector<uint64_t> pair_links;
  for (int i = 0; i < n_robots; ++i)
    for (int j = i + 1; j < n_robots; ++j) {
      const double dx = (double)robots[i].base_tf[3] - robots[j].base_tf[3];
      const double dy = (double)robots[i].base_tf[7] - robots[j].base_tf[7];
      const double dz = (double)robots[i].base_tf[11] - robots[j].base_tf[11];
      const double dist = std::sqrt(dx * dx + dy * dy + dz * dz);
      uint64_t mask = 0;
      for (int a = 0; a < kMaxLinks; ++a)
        for (int b = 0; b < kMaxLinks; ++b) {
          const double ra = link_reach[(size_t)model_of[i] * kMaxLinks + a],
                       rb = link_reach[(size_t)model_of[j] * kMaxLinks + b];
          if (ra >= 0 && rb >= 0 && dist <= ra + rb) mask |= 1ull << (a * kMaxLinks + b);
        }
      if (mask) {
        pairs.push_back(i);
        pairs.push_back(j);
        pair_links.push_back(mask);
      }
    }
  const int n_pairs = (int)pair_links.size();
  if (pairs.empty()) pairs.push_back(0), pairs.push_back(0), pair_links.push_back(0);  // placeholder

  Blob blob;
  size_t o_model = blob.add(model_of.data(), sizeof(int32_t) * n_robots);
  size_t o_qoff = blob.add(q_off.data(), sizeof(int32_t) * n_robots);
  size_t o_sout = blob.add(s_out.data(), sizeof(int32_t) * n_robots);
  size_t o_base = blob.add(base.data(), sizeof(float) * base.size());
  size_t o_nj = blob.add(nj.data(), sizeof(int32_t) * M);
  size_t o_dh = blob.add(dh.data(), sizeof(float4) * dh.size());
  size_t o_th = blob.add(th.data(), sizeof(float) * th.size());
  // order in which the tile kernel's waves claim the links of an arm: the
  // links with the most spheres (the longest fine tests) first
  std::vector<int32_t> link_order((size_t)M * kMaxLinks);
  for (int m = 0; m < M; ++m) {
    const int32_t *ls = &link_start[(size_t)m * (kMaxLinks + 1)];
    int32_t *ord = &link_order[(size_t)m * kMaxLinks];
    std::iota(ord, ord + kMaxLinks, 0);
    std::stable_sort(ord, ord + kMaxLinks, [&](int a, int b) { return ls[a + 1] - ls[a] > ls[b + 1] - ls[b]; });
  }
  size_t o_ls = blob.add(link_start.data(), sizeof(int32_t) * link_start.size());
  size_t o_lord = blob.add(link_order.data(), sizeof(int32_t) * link_order.size());
  size_t o_fine = blob.add(fine.data(), sizeof(float4) * fine.size());
  size_t o_fsrc = blob.add(fine_src.data(), sizeof(int32_t) * fine_src.size());
  size_t o_coarse = blob.add(coarse.data(), sizeof(float4) * coarse.size());
  size_t o_es = blob.add(env_s.data(), sizeof(float4) * env_s.size());
  size_t o_eb = blob.add(env_b.data(), sizeof(float4) * env_b.size());
  size_t o_lists = blob.add(lists.data(), sizeof(int32_t) * lists.size());
  size_t o_rows = blob.add(rows.data(), sizeof(float4) * rows.size());
  size_t o_robs = blob.add(row_obs.data(), sizeof(int32_t) * row_obs.size());
  size_t o_crows = blob.add(crows.data(), sizeof(float4) * crows.size());
  size_t o_pairs = blob.add(pairs.data(), sizeof(int32_t) * pairs.size());
  size_t o_plinks = blob.add(pair_links.data(), sizeof(uint64_t) * pair_links.size());
  std::vector<float> qlo_all, qhi_all;
  for (int r = 0; r < n_robots; ++r)
    for (int j = 0; j < robots[r].n_joints; ++j) {
      qlo_all.push_back(robots[r].q_lo[j]);
      qhi_all.push_back(robots[r].q_hi[j]);
    }
  size_t o_qlo = blob.add(qlo_all.data(), sizeof(float) * qlo_all.size());
  size_t o_qhi = blob.add(qhi_all.data(), sizeof(float) * qhi_all.size());

  mrpop_scene *sc = new mrpop_scene();
  sc->ctx = ctx;
  hipError_t e = hipSetDevice(ctx->device);
  if (e == hipSuccess) e = hipMalloc(&sc->blob, blob.host.size());
  if (e != hipSuccess) {
    delete sc;
    return hip_fail(ctx, e, "hipMalloc(scene)");
  }
  sc->blob_bytes = blob.host.size();
  e = hipMemcpy(sc->blob, blob.host.data(), blob.host.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    hipFree(sc->blob);
    delete sc;
    return hip_fail(ctx, e, "hipMemcpy(scene)");
  }
  auto at = [&](size_t off) { return (void *)((unsigned char *)sc->blob + off); };
  SceneDev &d = sc->dev;
  d.n_robots = n_robots;
  d.dof = dof;
  d.homogeneous = homog ? 1 : 0;
  d.total_spheres = S;
  d.model = (const int32_t *)at(o_model);
  d.q_off = (const int32_t *)at(o_qoff);
  d.s_out = (const int32_t *)at(o_sout);
  d.base = (const float *)at(o_base);
  d.n_models = M;
  d.sph_stride = sph_stride;
  d.nj = (const int32_t *)at(o_nj);
  d.dh = (const float4 *)at(o_dh);
  d.theta_off = (const float *)at(o_th);
  d.link_start = (const int32_t *)at(o_ls);
  d.link_order = (const int32_t *)at(o_lord);
  d.fine = (const float4 *)at(o_fine);
  d.fine_src = (const int32_t *)at(o_fsrc);
  d.coarse = (const float4 *)at(o_coarse);
  d.n_env_spheres = env->n_spheres;
  d.n_env_boxes = env->n_boxes;
  d.env_s = (const float4 *)at(o_es);
  d.env_b = (const float4 *)at(o_eb);
  d.origin = float3{(float)org[0], (float)org[1], (float)org[2]};
  d.link_lists = (const int32_t *)at(o_lists);
  d.rows = (const float4 *)at(o_rows);
  d.row_obs = (const int32_t *)at(o_robs);
  d.crows = (const float4 *)at(o_crows);
  d.n_clusters = (int32_t)std::min<int64_t>(NC, INT32_MAX);
  d.n_pairs = n_pairs;
  d.pair_links = (const uint64_t *)at(o_plinks);
  d.pairs = (const int32_t *)at(o_pairs);
  d.q_lo = (const float *)at(o_qlo);
  d.q_hi = (const float *)at(o_qhi);
  sc->h_robots.resize(n_robots);
  for (int r = 0; r < n_robots; ++r) {
    const mrpop_robot &rb = robots[r];
    HostRobot &h = sc->h_robots[r];
    h.n_joints = rb.n_joints;
    h.dh.assign(rb.dh, rb.dh + 4 * rb.n_joints);
    h.q_lo.assign(rb.q_lo, rb.q_lo + rb.n_joints);
    h.q_hi.assign(rb.q_hi, rb.q_hi + rb.n_joints);
    h.base.assign(rb.base_tf, rb.base_tf + 12);
    h.xyzr.assign(rb.sphere_xyzr, rb.sphere_xyzr + 4 * rb.n_spheres);
    h.link.assign(rb.sphere_link, rb.sphere_link + rb.n_spheres);
  }
  if (env->n_spheres) sc->h_env_s.assign(env->spheres, env->spheres + 4 * (size_t)env->n_spheres);
  if (env->n_boxes) sc->h_env_b.assign(env->boxes, env->boxes + 6 * (size_t)env->n_boxes);
  sc->n_robots = n_robots;
  sc->dof = dof;
  sc->total_spheres = S;
  sc->q_lo.resize(dof);
  sc->q_hi.resize(dof);
  sc->nj.resize(n_robots);
  for (int r = 0; r < n_robots; ++r) {
    sc->nj[r] = robots[r].n_joints;
    for (int j = 0; j < robots[r].n_joints; ++j) {
      sc->q_lo[q_off[r] + j] = robots[r].q_lo[j];
      sc->q_hi[q_off[r] + j] = robots[r].q_hi[j];
    }
  }
  *out = sc;
  return MRPOP_OK;
}

void mrpop_scene_destroy(mrpop_scene *scene) {
  if (!scene) return;
  for (mrpop_scene *a : scene->arm_cache) mrpop_scene_destroy(a);
  scene->arm_cache.clear();
  if (scene->blob) {
    hipSetDevice(scene->ctx->device);
    hipFree(scene->blob);
  }
  delete scene;
}

mrpop_status mrpop_scene_set_env(mrpop_scene *scene, const mrpop_env *env) {
  if (!scene) return fail(nullptr, MRPOP_E_INVALID_ARG, "scene_set_env: scene is NULL");
  mrpop_ctx *ctx = scene->ctx;
  if (!env) return fail(ctx, MRPOP_E_INVALID_ARG, "scene_set_env: env is NULL");
  // the same arms, from the scene's host copies
  std::vector<mrpop_robot> rb(scene->h_robots.size());
  for (size_t r = 0; r < rb.size(); ++r) {
    const HostRobot &h = scene->h_robots[r];
    rb[r] = mrpop_robot{h.n_joints, h.dh.data(), h.q_lo.data(), h.q_hi.data(), h.base.data(),
                        (int32_t)(h.xyzr.size() / 4), h.link.data(), h.xyzr.data()};
  }
  mrpop_scene *fresh = nullptr;
  const mrpop_status st = mrpop_scene_create(ctx, rb.data(), (int32_t)rb.size(), env, &fresh);
  if (st != MRPOP_OK) return st;
  const int32_t mode = scene->dev.tile_mode;
  std::swap(*scene, *fresh);  // fresh now holds the old device copy
  scene->dev.tile_mode = mode;
  mrpop_scene_destroy(fresh);
  return MRPOP_OK;
}

int32_t mrpop_scene_dof(const mrpop_scene *scene) { return scene ? scene->dof : 0; }
int32_t mrpop_scene_total_spheres(const mrpop_scene *scene) { return scene ? scene->total_spheres : 0; }
int32_t mrpop_scene_obstacle_clusters(const mrpop_scene *scene) { return scene ? scene->dev.n_clusters : 0; }

mrpop_status mrpop_scene_set_tile_mode(mrpop_scene *scene, int32_t mode) {
  if (!scene) return MRPOP_E_INVALID_ARG;
  if (mode != MRPOP_TILE_AUTO && mode != MRPOP_TILE_LDS && mode != MRPOP_TILE_SCALAR)
    return fail(scene->ctx, MRPOP_E_INVALID_ARG, "scene_set_tile_mode: unknown mode");
  scene->dev.tile_mode = mode;
  return MRPOP_OK;
}

int32_t mrpop_scene_tile_mode(const mrpop_scene *scene) { return scene ? scene->dev.tile_mode : -1; }

// ---------------------------------------------------------------------------
// FK and validation
// ---------------------------------------------------------------------------

mrpop_status mrpop_fk_spheres(mrpop_ctx *ctx, const mrpop_scene *scene, const float *q, int64_t n_cfg,
                              float *out_xyzr, void *stream) {
  if (!ctx) return fail(nullptr, MRPOP_E_INVALID_ARG, "fk_spheres: ctx is NULL");
  if (!scene || scene->ctx != ctx) return fail(ctx, MRPOP_E_INVALID_ARG, "fk_spheres: scene not from this ctx");
  if (n_cfg < 0) return fail(ctx, MRPOP_E_INVALID_ARG, "fk_spheres: n_cfg < 0");
  if (n_cfg == 0) return MRPOP_OK;
  if (!q || !out_xyzr) return fail(ctx, MRPOP_E_INVALID_ARG, "fk_spheres: NULL buffer");
  hipError_t e = hipSetDevice(ctx->device);
  if (e == hipSuccess) e = launch_fk_spheres(scene->dev, q, n_cfg, out_xyzr, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "fk_spheres launch");
  return MRPOP_OK;
}

// Argument checks shared by both validation entry points (the message names
// the entry point); MRPOP_OK with *done set when there is nothing to do.
static mrpop_status validate_args(mrpop_ctx *ctx, const mrpop_scene *scene, const float *qa, const float *qb,
                                  int64_t n_edges, float resolution, const int32_t *n_states_opt,
                                  uint8_t *out_valid, mrpop_validate_stats *stats_opt, const char *who, bool *done) {
  *done = false;
  if (!ctx) return fail(nullptr, MRPOP_E_INVALID_ARG, std::string(who) + ": ctx is NULL");
  if (!scene || scene->ctx != ctx) return fail(ctx, MRPOP_E_INVALID_ARG, std::string(who) + ": scene not from this ctx");
  if (n_edges < 0) return fail(ctx, MRPOP_E_INVALID_ARG, std::string(who) + ": n_edges < 0");
  if (!n_states_opt && !(resolution > 0.f && std::isfinite(resolution)))
    return fail(ctx, MRPOP_E_INVALID_ARG, std::string(who) + ": resolution must be finite and > 0");
  if (stats_opt) std::memset(stats_opt, 0, sizeof(*stats_opt));
  if (n_edges == 0) {
    *done = true;
    return MRPOP_OK;
  }
  if (!qa || !qb || !out_valid) return fail(ctx, MRPOP_E_INVALID_ARG, std::string(who) + ": NULL buffer");
  return MRPOP_OK;
}

// The launch's counters (in ws) into stats_opt; waits for the stream.
static mrpop_status validate_stats(mrpop_ctx *ctx, const ValidateScratch &ws, hipStream_t s,
                                   mrpop_validate_stats *stats_opt, const char *who) {
  uint64_t c[16];
  hipError_t e = hipMemcpyAsync(c, ws.counters, sizeof(c), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(ctx, e, who);
  stats_opt->edge_states = (int64_t)c[1];
  stats_opt->states_checked = (int64_t)c[2];
  stats_opt->tiles = (int64_t)c[3];
  stats_opt->nonfinite_edges = (int64_t)c[4];
  stats_opt->edges_invalid = (int64_t)c[5];
  for (int i = 0; i < 8; ++i) stats_opt->work[i] = (int64_t)c[8 + i];
  if (c[6]) return fail(ctx, MRPOP_E_INVALID_ARG, std::string(who) + ": an edge has too many states");
  return MRPOP_OK;
}

mrpop_status mrpop_validate_edges(mrpop_ctx *ctx, const mrpop_scene *scene, const float *qa, const float *qb,
                                  int64_t n_edges, float resolution, const int32_t *n_states_opt,
                                  uint8_t *out_valid, mrpop_validate_stats *stats_opt, void *stream) {
  bool done = false;
  mrpop_status st = validate_args(ctx, scene, qa, qb, n_edges, resolution, n_states_opt, out_valid, stats_opt,
                                  "validate_edges", &done);
  if (st != MRPOP_OK || done) return st;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  void *ws_base = nullptr;
  st = scratch_slot(ctx, 0, validate_scratch_bytes(n_edges), &ws_base);
  if (st != MRPOP_OK) return st;
  ValidateScratch ws = validate_scratch_layout(ws_base, n_edges);
  hipStream_t s = (hipStream_t)stream;
  e = launch_validate(scene->dev, qa, qb, n_edges, resolution, n_states_opt, out_valid, ws, s, profile_slot(ctx),
                      ctx->profiling ? ctx->prof_totals : nullptr, &ctx->last_grid, &ctx->last_block);
  if (e != hipSuccess) return hip_fail(ctx, e, "validate_edges launch");
  if (stats_opt) return validate_stats(ctx, ws, s, stats_opt, "validate_edges stats");
  return MRPOP_OK;
}

static_assert(MRPOP_COUNTED_MAX_EDGES == kFusedMaxEdges, "one-launch batch limit");

mrpop_status mrpop_validate_counted(mrpop_ctx *ctx, const mrpop_scene *scene, const float *qa, const float *qb,
                                    int64_t n_edges, const int32_t *n_states, uint8_t *out_valid,
                                    mrpop_validate_stats *stats_opt, void *stream) {
  bool done = false;
  mrpop_status st = validate_args(ctx, scene, qa, qb, n_edges, 0.f, n_states, out_valid, stats_opt,
                                  "validate_counted", &done);
  if (st != MRPOP_OK || done) return st;
  if (!n_states) return fail(ctx, MRPOP_E_INVALID_ARG, "validate_counted: n_states is NULL");
  if (n_edges > MRPOP_COUNTED_MAX_EDGES)
    return fail(ctx, MRPOP_E_INVALID_ARG, "validate_counted: more than MRPOP_COUNTED_MAX_EDGES edges");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  void *ws_base = nullptr;
  st = scratch_slot(ctx, 0, validate_scratch_bytes(n_edges), &ws_base);
  if (st != MRPOP_OK) return st;
  ValidateScratch ws = validate_scratch_layout(ws_base, n_edges);
  uint32_t *arrived = nullptr, *flags = nullptr, token = 0;
  e = small_launch_state(ctx, &arrived, &flags, &token);
  if (e != hipSuccess) return hip_fail(ctx, e, "validate_counted state");
  ws.flags = flags;
  hipStream_t s = (hipStream_t)stream;
  e = launch_validate_small(scene->dev, qa, qb, n_edges, n_states, out_valid, ws, arrived, token, s, profile_slot(ctx),
                            ctx->profiling ? ctx->prof_totals : nullptr, &ctx->last_grid, &ctx->last_block);
  if (e != hipSuccess) return hip_fail(ctx, e, "validate_counted launch");
  if (stats_opt) return validate_stats(ctx, ws, s, stats_opt, "validate_counted stats");
  return MRPOP_OK;
}

mrpop_status mrpop_tuner_configure(const char *cache_file, int32_t enable) {
  if (enable != 0 && enable != 1) return fail(nullptr, MRPOP_E_INVALID_ARG, "tuner_configure: enable must be 0 or 1");
  tuner_configure(cache_file, enable != 0);
  return MRPOP_OK;
}

int32_t mrpop_tuner_entries(void) { return tuner_entries(); }

mrpop_status mrpop_validate_edges_noalloc(mrpop_ctx *ctx, const mrpop_scene *scene, const float *qa,
                                          const float *qb, int64_t n_edges, float resolution,
                                          const int32_t *n_states_opt, uint8_t *out_valid,
                                          mrpop_validate_stats *stats_opt, void *stream) {
  bool done = false;
  mrpop_status st = validate_args(ctx, scene, qa, qb, n_edges, resolution, n_states_opt, out_valid, stats_opt,
                                  "validate_edges_noalloc", &done);
  if (st != MRPOP_OK || done) return st;
  if (n_edges > MRPOP_NOALLOC_MAX_EDGES || validate_scratch_bytes(n_edges) > kNoAllocScratchBytes)
    return fail(ctx, MRPOP_E_INVALID_ARG, "validate_edges_noalloc: more than MRPOP_NOALLOC_MAX_EDGES edges");
  void *base = noalloc_scratch_ptr(ctx->device);
  if (!base) return fail(ctx, MRPOP_E_DEVICE, "validate_edges_noalloc: no scratch address for the device");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  // every launch of the general path writes the scratch words it later reads
  // (counts, offsets, flags, counters, partial sums), so nothing is cleared
  ValidateScratch ws = validate_scratch_layout(base, n_edges);
  hipStream_t s = (hipStream_t)stream;
  e = launch_validate(scene->dev, qa, qb, n_edges, resolution, n_states_opt, out_valid, ws, s, nullptr, nullptr,
                      nullptr, nullptr, /*may_tune=*/false);
  if (e != hipSuccess) return hip_fail(ctx, e, "validate_edges_noalloc launch");
  if (stats_opt) return validate_stats(ctx, ws, s, stats_opt, "validate_edges_noalloc stats");
  return MRPOP_OK;
}

}  // extern "C"
