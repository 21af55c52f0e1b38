// Composite edge validation: state counts, prefix scan, and the tile kernel.
//
// An edge (q_a, q_b) is checked at n discretised states (paper, Sec.
// "Multi-Thread Reassignment for Collision Checking").  The states of all
// edges form one global list (exclusive prefix sum of the per-edge counts);
// persistent workgroups pull tiles of 64 consecutive list positions from an
// atomic queue.
//
// Mapping: one lane per state.  A workgroup has W = min(R, 8) waves; wave w
// runs arms w, w + W, ... over the tile's 64 states, so every wave works on
// one arm at a time and all of that arm's model data is wave-uniform (scalar
// loads), while consecutive states of an edge sit in neighbouring lanes and
// take the same branches.  Per arm:
//   1. compose all link frames (modified DH) in registers and publish the
//      links' coarse centres in LDS;
//   2. obstacle by obstacle, one 64-byte scalar row holds everything needed
//      to test the obstacle (sphere, or a box's bounding sphere) against all
//      eight coarse link spheres in expanded form (three FMAs and a compare
//      each); one wave-wide vote per obstacle skips it when no lane flags it;
//   3. only for flagged (link, obstacle) pairs: the exact link-box distance,
//      then the link's fine spheres.
// After a barrier, the arm pairs that can reach each other are split over the
// waves: coarse link-link tests from the LDS centres, and for flagged link
// pairs the two frames are rebuilt and the fine spheres tested.
// A collision marks the edge in a flag word and marks all of the edge's lanes
// of the tile in an LDS mask, which the other waves read as they go; states of
// an edge already marked by an earlier tile are skipped.
#include <algorithm>

#include "device_common.h"

namespace mrpop {

constexpr int kScanThreads = 1024;
constexpr int kScanItems = 4;
constexpr int kScanChunk = kScanThreads * kScanItems;

enum : uint32_t { kFlagHit = 1u, kFlagNonFinite = 2u, kFlagTooLong = 4u };

static int64_t scan_blocks(int64_t n) { return (n + kScanChunk - 1) / kScanChunk; }

size_t validate_scratch_bytes(int64_t n_edges) {
  size_t b = 0;
  auto add = [&](size_t n) {
    b = (b + 255) & ~size_t(255);
    b += n;
  };
  add(sizeof(int32_t) * n_edges);
  add(sizeof(int64_t) * (n_edges + 1));
  add(sizeof(uint32_t) * n_edges);
  add(sizeof(uint64_t) * 16);
  add(sizeof(int64_t) * (scan_blocks(n_edges) + 1));
  add(sizeof(uint64_t) * kPartialSlots * kMaxGrid);
  add(sizeof(int32_t) * kTileFirstCap);
  return b + 256;
}

ValidateScratch validate_scratch_layout(void *base, int64_t n_edges) {
  size_t b = 0;
  auto take = [&](size_t n) {
    b = (b + 255) & ~size_t(255);
    void *p = (unsigned char *)base + b;
    b += n;
    return p;
  };
  ValidateScratch w;
  w.n_states = (int32_t *)take(sizeof(int32_t) * n_edges);
  w.offsets = (int64_t *)take(sizeof(int64_t) * (n_edges + 1));
  w.flags = (uint32_t *)take(sizeof(uint32_t) * n_edges);
  w.counters = (uint64_t *)take(sizeof(uint64_t) * 16);
  w.block_sums = (int64_t *)take(sizeof(int64_t) * (scan_blocks(n_edges) + 1));
  w.partials = (uint64_t *)take(sizeof(uint64_t) * kPartialSlots * kMaxGrid);
  w.tile_first = (int32_t *)take(sizeof(int32_t) * kTileFirstCap);
  return w;
}

// ---------------------------------------------------------------------------
// 1. per-edge state counts
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void count_states_kernel(const float *__restrict__ qa, const float *__restrict__ qb,
                                                           int64_t n_edges, int dof, float res,
                                                           const int32_t *__restrict__ n_opt,
                                                           int32_t *__restrict__ n_out, uint32_t *__restrict__ flags) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_edges) return;
  const float *a = qa + e * dof, *b = qb + e * dof;
  bool finite = true;
  float linf = 0.f;
  for (int j = 0; j < dof; ++j) {
    const float x = a[j], y = b[j];
    finite = finite && isfinite(x) && isfinite(y);
    linf = fmaxf(linf, fabsf(y - x));
  }
  int32_t n = 0;
  uint32_t f = 0;
  if (!finite) {
    f = kFlagNonFinite;
  } else if (n_opt) {
    const int32_t v = n_opt[e];
    if (v < 1 || v > MRPOP_MAX_STATES_PER_EDGE) f = kFlagTooLong;
    else n = v;
  } else if (linf == 0.f) {
    n = 1;
  } else {
    const float ratio = linf / res;  // correctly rounded single-precision division
    if (!(ratio <= (float)(MRPOP_MAX_STATES_PER_EDGE - 1))) f = kFlagTooLong;
    else n = 1 + (int32_t)ceilf(ratio);
  }
  n_out[e] = n;
  flags[e] = f;
}

// ---------------------------------------------------------------------------
// 2. exclusive prefix sum of the counts (three passes)
// ---------------------------------------------------------------------------

// Exclusive scan of one value per thread across the block; returns the
// exclusive prefix and writes the block total.
__device__ int64_t block_exclusive_scan(int64_t v, int64_t *total) {
  __shared__ int64_t wave_sums[kScanThreads / kWave];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  int64_t x = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int64_t y = __shfl_up(x, d, kWave);
    if (lane >= d) x += y;
  }
  if (lane == kWave - 1) wave_sums[wid] = x;
  __syncthreads();
  if (wid == 0) {
    const int nw = blockDim.x / kWave;
    int64_t w = lane < nw ? wave_sums[lane] : 0;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      const int64_t y = __shfl_up(w, d, kWave);
      if (lane >= d) w += y;
    }
    if (lane < nw) wave_sums[lane] = w;  // inclusive
  }
  __syncthreads();
  const int64_t wave_prefix = wid > 0 ? wave_sums[wid - 1] : 0;
  *total = wave_sums[blockDim.x / kWave - 1];
  __syncthreads();
  return wave_prefix + x - v;
}

__global__ __launch_bounds__(kScanThreads) void scan_partials_kernel(const int32_t *__restrict__ n, int64_t n_edges,
                                                                     int64_t *__restrict__ block_sums) {
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n_edges) s += n[base + i];
  int64_t total;
  block_exclusive_scan(s, &total);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// Single block: exclusive scan of the block sums; publishes the total and
// resets the work counters for the tile kernel.
__global__ __launch_bounds__(kScanThreads) void scan_top_kernel(int64_t *__restrict__ block_sums, int64_t nb,
                                                                uint64_t *__restrict__ counters) {
  int64_t carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += kScanThreads) {
    const int64_t i = b0 + threadIdx.x;
    const int64_t v = i < nb ? block_sums[i] : 0;
    int64_t total;
    const int64_t ex = block_exclusive_scan(v, &total);
    if (i < nb) block_sums[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) {
    block_sums[nb] = carry;
    counters[0] = 0;                    // tile queue
    counters[1] = (uint64_t)carry;      // total states
    for (int c = 2; c < 16; ++c) counters[c] = 0;
  }
}

// Writes the exclusive offsets and, for every tile of kWave list positions
// (below kTileFirstCap), the edge that holds the tile's first position.
__global__ __launch_bounds__(kScanThreads) void scan_apply_kernel(const int32_t *__restrict__ n, int64_t n_edges,
                                                                  const int64_t *__restrict__ block_sums,
                                                                  int64_t *__restrict__ offsets,
                                                                  int32_t *__restrict__ tile_first) {
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
  int64_t v[kScanItems], s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = base + i < n_edges ? n[base + i] : 0;
    s += v[i];
  }
  int64_t total;
  int64_t run = block_sums[blockIdx.x] + block_exclusive_scan(s, &total);
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n_edges) {
      offsets[base + i] = run;
      // tiles whose first position falls inside this edge: [run, run + v)
      for (int64_t tl = (run + kWave - 1) / kWave; tl * kWave < run + v[i] && tl < kTileFirstCap; ++tl)
        tile_first[tl] = (int32_t)(base + i);
    }
    run += v[i];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) offsets[n_edges] = block_sums[gridDim.x];
}

// ---------------------------------------------------------------------------
// 3. tile kernel
// ---------------------------------------------------------------------------

// Last edge e with offsets[e] <= s (skips empty edges).
__device__ __forceinline__ int64_t find_edge(const int64_t *__restrict__ off, int64_t n_edges, int64_t s) {
  int64_t lo = 0, hi = n_edges - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (off[mid] <= s) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Work actually executed by one lane (for the algorithmic flop count): kinematic
// chains, coarse link centres placed, coarse link-obstacle sphere tests
// (environment spheres and box bounding spheres), exact link-box tests,
// coarse link-link tests, and fine sphere tests by kind.
struct WorkCount {
  uint32_t chains = 0, links = 0, env_tests = 0, box_exact = 0, rr_coarse = 0, fine_s = 0, fine_b = 0, fine_rr = 0;
};

// Per-lane view of the state being checked.
struct LaneState {
  const float *qa, *qb;  // the edge's endpoints (composite rows)
  float t;               // interpolation parameter k / (n - 1)
  bool last;             // k == n - 1: the state is exactly qb
};

__device__ __forceinline__ float joint_value(const LaneState &ls, int idx) {
  const float a = ls.qa[idx], b = ls.qb[idx];
  return ls.last ? b : fmaf(ls.t, b - a, a);
}

__device__ __forceinline__ Frame base_frame(const SceneDev &sc, int r) {
  const cptr<float> p = as_const(sc.base) + 12 * r;
  Frame f;
  f.r00 = p[0]; f.r01 = p[1]; f.r02 = p[2]; f.t0 = p[3];
  f.r10 = p[4]; f.r11 = p[5]; f.r12 = p[6]; f.t1 = p[7];
  f.r20 = p[8]; f.r21 = p[9]; f.r22 = p[10]; f.t2 = p[11];
  return f;
}

// Frame of link `link` of arm r (model m) at the lane's state, rebuilt from
// the joint values.
__device__ Frame frame_at(const SceneDev &sc, int r, int m, const LaneState &ls, int link) {
  Frame F = base_frame(sc, r);
  const int q0 = as_const(sc.q_off)[r];
  for (int j = 1; j <= link; ++j)
    joint_step(F, ld4(as_const(sc.dh), m * kMaxJoints + j - 1),
               joint_value(ls, q0 + j - 1) + as_const(sc.theta_off)[m * kMaxJoints + j - 1]);
  return F;
}

__device__ __forceinline__ uint64_t dead_mask(const unsigned long long *d) {
  return __hip_atomic_load(d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

constexpr int kRowUsed = 3 + kMaxLinks;  // -2 o (3 floats), w_l for every link

struct Row {
  float v[kRowUsed];
};

// Scene data the tile kernel reads inside its loops: obstacle rows, box
// corners, fine spheres, link ranges and coarse radii.  STAGED: copies in
// LDS, made once per persistent workgroup (the scalar cache starts cold at
// every launch, and a miss costs far more than the tests one row feeds).
// Otherwise: the scene arrays themselves, read with scalar loads.
template <bool STAGED>
struct Src;

template <>
struct Src<true> {
  const float *srows, *brows;  // [M][N][kRowFloats]
  const float4 *boxes;         // [Nb][2]
  const float4 *fine;          // [M][sph_stride]
  const int32_t *lstart;       // [M][kMaxLinks + 1]
  const float *crad;           // [M][kMaxLinks]
  int ns, nb, stride;
  __device__ Row srow(int m, int k) const { return row(srows + ((int64_t)m * ns + k) * kRowFloats); }
  __device__ Row brow(int m, int k) const { return row(brows + ((int64_t)m * nb + k) * kRowFloats); }
  __device__ static Row row(const float *p) {
    Row r;
#pragma unroll
    for (int i = 0; i < kRowUsed; ++i) r.v[i] = p[i];
    return r;
  }
  __device__ float4 box(int i) const { return boxes[i]; }
  __device__ float4 sph(int m, int i) const { return fine[m * stride + i]; }
  __device__ int ls(int m, int l) const { return lstart[m * (kMaxLinks + 1) + l]; }
  __device__ float rad(int m, int l) const { return crad[m * kMaxLinks + l]; }
};

template <>
struct Src<false> {
  cptr<float> srows, brows;
  cptr<float4> boxes, fine, coarse;
  cptr<int32_t> lstart;
  int ns, nb, stride;
  __device__ Row srow(int m, int k) const { return row(srows + ((int64_t)m * ns + k) * kRowFloats); }
  __device__ Row brow(int m, int k) const { return row(brows + ((int64_t)m * nb + k) * kRowFloats); }
  __device__ static Row row(cptr<float> p) {
    Row r;
#pragma unroll
    for (int i = 0; i < kRowUsed; ++i) r.v[i] = p[i];
    return r;
  }
  __device__ float4 box(int i) const { return ld4(boxes, i); }
  __device__ float4 sph(int m, int i) const { return ld4(fine, (int64_t)m * stride + i); }
  __device__ int ls(int m, int l) const { return lstart[m * (kMaxLinks + 1) + l]; }
  __device__ float rad(int m, int l) const { return ld4(coarse, m * kMaxLinks + l).w; }
};

// LDS floats needed to stage a scene (0 when it does not fit the budget).
__host__ __device__ inline size_t staged_floats(const SceneDev &sc) {
  const size_t M = sc.n_models;
  return M * (size_t)(sc.n_env_spheres + sc.n_env_boxes) * kRowFloats + (size_t)sc.n_env_boxes * 8 +
         M * (size_t)sc.sph_stride * 4 + M * (kMaxLinks + 1) + M * kMaxLinks;
}

template <bool STAGED>
__device__ Src<STAGED> make_src(const SceneDev &sc, float *stage);

template <>
__device__ Src<true> make_src<true>(const SceneDev &sc, float *stage) {
  // copy once per workgroup, coalesced
  const int M = sc.n_models;
  Src<true> s;
  s.ns = sc.n_env_spheres;
  s.nb = sc.n_env_boxes;
  s.stride = sc.sph_stride;
  float *p = stage;
  s.srows = p;
  const int n_s = M * s.ns * kRowFloats;
  for (int i = threadIdx.x; i < n_s; i += blockDim.x) p[i] = sc.sph_rows[i];
  p += n_s;
  s.brows = p;
  const int n_b = M * s.nb * kRowFloats;
  for (int i = threadIdx.x; i < n_b; i += blockDim.x) p[i] = sc.box_rows[i];
  p += n_b;
  s.boxes = (const float4 *)p;
  for (int i = threadIdx.x; i < 2 * s.nb; i += blockDim.x) ((float4 *)p)[i] = sc.env_b[i];
  p += 8 * s.nb;
  s.fine = (const float4 *)p;
  for (int i = threadIdx.x; i < M * s.stride; i += blockDim.x) ((float4 *)p)[i] = sc.fine[i];
  p += 4 * M * s.stride;
  s.lstart = (const int32_t *)p;
  for (int i = threadIdx.x; i < M * (kMaxLinks + 1); i += blockDim.x) ((int32_t *)p)[i] = sc.link_start[i];
  p += M * (kMaxLinks + 1);
  s.crad = p;
  for (int i = threadIdx.x; i < M * kMaxLinks; i += blockDim.x) p[i] = sc.coarse[i].w;
  __syncthreads();
  return s;
}

template <>
__device__ Src<false> make_src<false>(const SceneDev &sc, float *) {
  Src<false> s;
  s.srows = as_const(sc.sph_rows);
  s.brows = as_const(sc.box_rows);
  s.boxes = as_const(sc.env_b);
  s.fine = as_const(sc.fine);
  s.coarse = as_const(sc.coarse);
  s.lstart = as_const(sc.link_start);
  s.ns = sc.n_env_spheres;
  s.nb = sc.n_env_boxes;
  s.stride = sc.sph_stride;
  return s;
}

__device__ __forceinline__ float link_test(const float3 &c, float c2, const Row &row, int l) {
  return fmaf(c.z, row.v[2], fmaf(c.y, row.v[1], fmaf(c.x, row.v[0], c2))) + row.v[3 + l];
}

// Environment test of arm model m at every lane's state.  F: link frames,
// c/c2: coarse centres and their squared norms for links 0..kMaxLinks-1 (links
// the model lacks have row entries that never pass).  Returns true for lanes
// whose state collides.
template <bool STAGED>
__device__ bool arm_env(const SceneDev &sc, const Src<STAGED> &src, int m, const Frame (&F)[kMaxLinks],
                        const float3 (&c)[kMaxLinks], const float (&c2)[kMaxLinks], int n_links, bool live,
                        WorkCount &wc) {
  const cptr<float4> env_s = as_const(sc.env_s);
  bool hit = false;
  int ls[kMaxLinks + 1];
#pragma unroll
  for (int l = 0; l <= kMaxLinks; ++l) ls[l] = src.ls(m, l);
  // environment spheres; rows are fetched one obstacle ahead
  Row nxt;
  if (src.ns > 0) nxt = src.srow(m, 0);
  for (int k = 0; k < src.ns; ++k) {
    const Row row = nxt;
    if (k + 1 < src.ns) nxt = src.srow(m, k + 1);
    uint64_t any = 0;
#pragma unroll
    for (int l = 0; l < kMaxLinks; ++l) any |= __ballot(link_test(c[l], c2[l], row, l) < 0.f);
    if (live) wc.env_tests += n_links;
    if ((any & __ballot(live)) == 0ull) continue;
    const float4 o = ld4(env_s, k);
#pragma unroll
    for (int l = 0; l < kMaxLinks; ++l) {
      if (live && link_test(c[l], c2[l], row, l) < 0.f) {
        for (int i = ls[l]; i < ls[l + 1]; ++i) {
          const float4 p = src.sph(m, i);
          const float3 w = apply(F[l], p.x, p.y, p.z);
          const float rr = p.w + o.w;
          ++wc.fine_s;
          if (dist2(w, o) < rr * rr) {
            hit = true;
            live = false;
            break;
          }
        }
      }
    }
  }
  // boxes: bounding-sphere filter, exact distance, then fine spheres
  if (src.nb > 0) nxt = src.brow(m, 0);
  for (int k = 0; k < src.nb; ++k) {
    const Row row = nxt;
    if (k + 1 < src.nb) nxt = src.brow(m, k + 1);
    uint64_t any = 0;
#pragma unroll
    for (int l = 0; l < kMaxLinks; ++l) any |= __ballot(link_test(c[l], c2[l], row, l) < 0.f);
    if (live) wc.env_tests += n_links;
    if ((any & __ballot(live)) == 0ull) continue;
    const float4 lo = src.box(2 * k), hi = src.box(2 * k + 1);
#pragma unroll
    for (int l = 0; l < kMaxLinks; ++l) {
      if (live && link_test(c[l], c2[l], row, l) < 0.f) {
        ++wc.box_exact;
        const float cr = src.rad(m, l);
        if (box_dist2(c[l], lo, hi) < cr * cr) {
          for (int i = ls[l]; i < ls[l + 1]; ++i) {
            const float4 p = src.sph(m, i);
            const float3 w = apply(F[l], p.x, p.y, p.z);
            ++wc.fine_b;
            if (box_dist2(w, lo, hi) < p.w * p.w) {
              hit = true;
              live = false;
              break;
            }
          }
        }
      }
    }
  }
  return hit;
}

// Arm pair (i, j) at the lane's state: coarse link-link tests on the
// published centres; flagged link pairs rebuild both frames and test the
// fine spheres.
template <bool STAGED>
__device__ bool pair_test(const SceneDev &sc, const Src<STAGED> &src, const float *cen, int lane, int i, int j,
                          const LaneState &ls, WorkCount &wc) {
  const int mi = as_const(sc.model)[i], mj = as_const(sc.model)[j];
  const int nji = as_const(sc.nj)[mi], njj = as_const(sc.nj)[mj];
  float3 cb[kMaxLinks];
  float rb[kMaxLinks], ra[kMaxLinks];
#pragma unroll
  for (int b = 0; b < kMaxLinks; ++b) {
    const float *p = cen + ((j * kMaxLinks + b) * 3) * kWave + lane;
    cb[b] = make_float3(p[0], p[kWave], p[2 * kWave]);
    rb[b] = b <= njj ? src.rad(mj, b) : -1.f;
    ra[b] = b <= nji ? src.rad(mi, b) : -1.f;
  }
  for (int a = 0; a <= nji; ++a) {
    if (ra[a] < 0.f) continue;
    const float *p = cen + ((i * kMaxLinks + a) * 3) * kWave + lane;
    const float3 ca = make_float3(p[0], p[kWave], p[2 * kWave]);
    uint64_t any = 0;
#pragma unroll
    for (int b = 0; b < kMaxLinks; ++b) {
      if (rb[b] < 0.f) continue;
      const float rs = ra[a] + rb[b];
      ++wc.rr_coarse;
      any |= __ballot(dist2(ca, cb[b]) < rs * rs);
    }
    if (any == 0ull) continue;
    bool have_a = false;
    Frame Fa;
    for (int b = 0; b <= njj; ++b) {
      const float rbb = src.rad(mj, b);
      if (rbb < 0.f) continue;
      const float *q = cen + ((j * kMaxLinks + b) * 3) * kWave + lane;
      const float3 cq = make_float3(q[0], q[kWave], q[2 * kWave]);
      const float rs = ra[a] + rbb;
      if (!(dist2(ca, cq) < rs * rs)) continue;
      if (!have_a) {
        Fa = frame_at(sc, i, mi, ls, a);
        have_a = true;
      }
      const Frame Fb = frame_at(sc, j, mj, ls, b);
      for (int x = src.ls(mi, a); x < src.ls(mi, a + 1); ++x) {
        const float4 pa = src.sph(mi, x);
        const float3 wa = apply(Fa, pa.x, pa.y, pa.z);
        for (int y = src.ls(mj, b); y < src.ls(mj, b + 1); ++y) {
          const float4 pb = src.sph(mj, y);
          const float3 wb = apply(Fb, pb.x, pb.y, pb.z);
          const float r2 = pa.w + pb.w;
          ++wc.fine_rr;
          if (dist2(wa, wb) < r2 * r2) return true;
        }
      }
    }
  }
  return false;
}

template <bool STAGED>
__global__ __launch_bounds__(kWave * kMaxWavesPerBlock) void validate_tiles_kernel(
    SceneDev sc, const float *__restrict__ qa, const float *__restrict__ qb, int64_t n_edges,
    const int64_t *__restrict__ off, const int32_t *__restrict__ tile_first, uint32_t *__restrict__ flags,
    uint64_t *__restrict__ counters, uint64_t *__restrict__ partials) {
  extern __shared__ float cen[];  // [R][kMaxLinks][3][64] published coarse centres, then staged scene data
  __shared__ unsigned long long s_cur, s_dead;
  const int lane = threadIdx.x & (kWave - 1);
  // wave index, marked wave-uniform so that per-arm data is read with scalar loads
  const int w = (int)__builtin_amdgcn_readfirstlane(threadIdx.x / kWave), W = blockDim.x / kWave;
  const int R = sc.n_robots;
  const int64_t total = (int64_t)counters[1];
  const int64_t n_tiles = (total + kWave - 1) / kWave;
  if ((int64_t)blockIdx.x >= n_tiles) {
    if (threadIdx.x < kPartialSlots) partials[(int64_t)blockIdx.x * kPartialSlots + threadIdx.x] = 0ull;
    return;
  }
  uint32_t checked = 0, tiles = 0;
  WorkCount wc;
  // The first tile of every workgroup is its block index; later ones come
  // from the shared queue, claimed one tile ahead so that the claim's latency
  // overlaps the current tile (device-wide atomics are slow on this chip,
  // whose eight XCDs do not share an L2).
  unsigned long long pending = 0;
  if (threadIdx.x == 0) {
    s_dead = 0ull;
    pending = (unsigned long long)gridDim.x + atomicAdd((unsigned long long *)&counters[0], 1ull);
  }
  const Src<STAGED> src = make_src<STAGED>(sc, cen + (size_t)R * kMaxLinks * 3 * kWave);
  int64_t tile = blockIdx.x;
  for (;;) {
    __syncthreads();
    if (tile >= n_tiles) break;
    if (w == 0) ++tiles;
    const int64_t s0 = tile * kWave;
    const int64_t s = s0 + lane;
    bool act = s < total;
    // edge of each lane: the tile starts in edge e0 and spans at most 64
    // consecutive edges; lane i holds off[e0 + i] and a binary search over
    // lanes finds the last edge starting at or before the lane's position
    const int64_t e0 = tile < kTileFirstCap ? (int64_t)as_const(tile_first)[tile] : find_edge(off, n_edges, s0);
    const int64_t ei = e0 + lane < n_edges ? e0 + lane : n_edges;
    const int64_t my_off = off[ei];
    int pos = 0;
#pragma unroll
    for (int step = kWave / 2; step > 0; step >>= 1) {
      const int cand = pos + step;
      const int64_t o = __shfl(my_off, cand, kWave);
      if (o <= s) pos = cand;
    }
    const int64_t e = e0 + pos;
    const int64_t e_start = __shfl(my_off, pos, kWave);
    int64_t e_end = __shfl(my_off, pos < kWave - 1 ? pos + 1 : pos, kWave);
    if (act && pos == kWave - 1) e_end = off[e + 1];  // active lanes have e < n_edges
    LaneState st{qa, qb, 0.f, false};
    uint64_t emask = 0;  // lanes of this tile on the same edge
    if (act) {
      const int64_t n = e_end - e_start;
      const int64_t k = s - e_start;
      st.qa = qa + e * sc.dof;
      st.qb = qb + e * sc.dof;
      st.last = n > 1 && k == n - 1;
      st.t = n > 1 ? (float)k / (float)(n - 1) : 0.f;
      const int lo = (int)((e_start > s0 ? e_start : s0) - s0);
      const int hi = (int)((e_end < s0 + kWave ? e_end : s0 + kWave) - s0);
      emask = (hi - lo >= 64 ? ~0ull : ((1ull << (hi - lo)) - 1ull)) << lo;
      if (load_relaxed(flags + e) != 0u) act = false;
    }
    if (act && w == 0) ++checked;
    bool hit = false;
    // environment, one arm per wave at a time
    for (int r = w; r < R; r += W) {
      const int m = as_const(sc.model)[r];
      const int nj = as_const(sc.nj)[m];
      const int q0 = as_const(sc.q_off)[r];
      // all joint values of the arm first, so that their loads overlap
      float qv[kMaxJoints];
      {
        float qa_v[kMaxJoints], qb_v[kMaxJoints];
#pragma unroll
        for (int j = 0; j < kMaxJoints; ++j) {
          const int idx = j < nj ? q0 + j : q0;
          qa_v[j] = st.qa[idx];
          qb_v[j] = st.qb[idx];
        }
#pragma unroll
        for (int j = 0; j < kMaxJoints; ++j) qv[j] = st.last ? qb_v[j] : fmaf(st.t, qb_v[j] - qa_v[j], qa_v[j]);
      }
      Frame F[kMaxLinks];
      float3 c[kMaxLinks];
      float c2[kMaxLinks];
      F[0] = base_frame(sc, r);
#pragma unroll
      for (int l = 1; l < kMaxLinks; ++l) {
        F[l] = F[l - 1];
        if (l <= nj)
          joint_step(F[l], ld4(as_const(sc.dh), m * kMaxJoints + l - 1),
                     qv[l - 1] + as_const(sc.theta_off)[m * kMaxJoints + l - 1]);
      }
      int n_links = 0;
#pragma unroll
      for (int l = 0; l < kMaxLinks; ++l) {
        const float4 cs = ld4(as_const(sc.coarse), m * kMaxLinks + l);
        c[l] = apply(F[l], cs.x, cs.y, cs.z);
        c2[l] = fmaf(c[l].z, c[l].z, fmaf(c[l].y, c[l].y, c[l].x * c[l].x));
        n_links += (l <= nj && cs.w >= 0.f) ? 1 : 0;
        if (l <= nj) {
          float *slot = cen + ((r * kMaxLinks + l) * 3) * kWave + lane;
          slot[0] = c[l].x;
          slot[kWave] = c[l].y;
          slot[2 * kWave] = c[l].z;
        }
      }
      const bool live = act && !hit && !((dead_mask(&s_dead) >> lane) & 1ull);
      if (live) {
        ++wc.chains;
        wc.links += n_links;
      }
      if (arm_env<STAGED>(sc, src, m, F, c, c2, n_links, live, wc)) {
        hit = true;
        atomicOr(&s_dead, (unsigned long long)emask);
      }
    }
    __syncthreads();
    // arm pairs that can reach each other
    for (int p = w; p < sc.n_pairs; p += W) {
      const int pi = as_const(sc.pairs)[2 * p], pj = as_const(sc.pairs)[2 * p + 1];
      const bool live = act && !hit && !((dead_mask(&s_dead) >> lane) & 1ull);
      if (live && pair_test<STAGED>(sc, src, cen, lane, pi, pj, st, wc)) {
        hit = true;
        atomicOr(&s_dead, (unsigned long long)emask);
      }
    }
    if (hit) flags[e] = kFlagHit;
    __syncthreads();
    if (threadIdx.x == 0) {
      // hand over the claimed tile and claim the next one; its result is not
      // needed before the next hand-over
      s_cur = pending;
      pending = (unsigned long long)gridDim.x + atomicAdd((unsigned long long *)&counters[0], 1ull);
      s_dead = 0ull;
    }
    __syncthreads();
    tile = (int64_t)uniform_u64(s_cur);
  }
  // workgroup totals of the work counters, one slot row per workgroup
  // (summed by the final kernel; no device-wide atomics)
  __shared__ unsigned long long s_part[kPartialSlots];
  if (threadIdx.x < kPartialSlots) s_part[threadIdx.x] = 0ull;
  __syncthreads();
  uint64_t v[kPartialSlots - 1] = {checked,      wc.chains, wc.links,  wc.env_tests, wc.box_exact,
                                   wc.rr_coarse, wc.fine_s, wc.fine_b, wc.fine_rr};
#pragma unroll
  for (int i = 0; i < kPartialSlots - 1; ++i)
    for (int d = kWave / 2; d > 0; d >>= 1) v[i] += __shfl_xor(v[i], d, kWave);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < kPartialSlots - 1; ++i) atomicAdd(&s_part[i], (unsigned long long)v[i]);
    if (w == 0) atomicAdd(&s_part[kPartialSlots - 1], (unsigned long long)tiles);
  }
  __syncthreads();
  if (threadIdx.x < kPartialSlots) partials[(int64_t)blockIdx.x * kPartialSlots + threadIdx.x] = s_part[threadIdx.x];
}

__global__ __launch_bounds__(256) void finalize_kernel(const uint32_t *__restrict__ flags, int64_t n_edges,
                                                       uint8_t *__restrict__ out, uint64_t *__restrict__ counters,
                                                       const uint64_t *__restrict__ partials, int n_partials,
                                                       uint64_t *__restrict__ totals) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.x == 0) {
    // column sums of the tile kernel's per-workgroup partials
    __shared__ unsigned long long col[kPartialSlots];
    if (threadIdx.x < kPartialSlots) col[threadIdx.x] = 0ull;
    __syncthreads();
    for (int i = 0; i < kPartialSlots; ++i) {
      uint64_t acc = 0;
      for (int b = threadIdx.x; b < n_partials; b += blockDim.x) acc += partials[(int64_t)b * kPartialSlots + i];
      for (int d = kWave / 2; d > 0; d >>= 1) acc += __shfl_xor(acc, d, kWave);
      if ((threadIdx.x & (kWave - 1)) == 0) atomicAdd(&col[i], (unsigned long long)acc);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      counters[2] = col[0];
      counters[3] = col[kPartialSlots - 1];
      for (int i = 1; i < kPartialSlots - 1; ++i) counters[7 + i] = col[i];
      if (totals) {
        totals[0] += col[0];
        totals[1] += counters[1];
        for (int i = 1; i < kPartialSlots - 1; ++i) totals[1 + i] += col[i];
      }
    }
  }
  uint32_t f = e < n_edges ? flags[e] : 0u;
  if (e < n_edges) out[e] = f == 0u ? 1 : 0;
  const uint64_t inval = __ballot(f != 0u), nonfin = __ballot((f & kFlagNonFinite) != 0u),
                 toolong = __ballot((f & kFlagTooLong) != 0u);
  if ((threadIdx.x & (kWave - 1)) == 0) {
    if (inval) atomicAdd((unsigned long long *)&counters[5], (unsigned long long)__popcll(inval));
    if (nonfin) atomicAdd((unsigned long long *)&counters[4], (unsigned long long)__popcll(nonfin));
    if (toolong) atomicAdd((unsigned long long *)&counters[6], (unsigned long long)__popcll(toolong));
  }
}

static int block_waves(int n_robots) { return n_robots < kMaxWavesPerBlock ? n_robots : kMaxWavesPerBlock; }

static size_t centre_lds_bytes(int n_robots) { return (size_t)n_robots * kMaxLinks * 3 * kWave * sizeof(float); }

// Dynamic LDS budget of the tile kernel: staging is used when the scene's
// copy fits next to the published centres.
constexpr size_t kLdsBudget = 150 * 1024;

static bool use_staged(const SceneDev &sc) {
  return centre_lds_bytes(sc.n_robots) + staged_floats(sc) * sizeof(float) <= kLdsBudget;
}

// Resident workgroups for a persistent launch (cached per arm count, staging
// and LDS size).
template <bool STAGED>
static int persistent_grid(int n_robots, size_t lds) {
  struct Key {
    int r;
    size_t lds;
    int grid;
  };
  static std::vector<Key> cache;
  for (const Key &k : cache)
    if (k.r == n_robots && k.lds == lds) return k.grid;
  int dev = 0, cus = 0, per = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, validate_tiles_kernel<STAGED>,
                                                     kWave * block_waves(n_robots), lds);
  const int grid = std::min(kMaxGrid, std::max(1, cus) * std::max(1, per));
  cache.push_back({n_robots, lds, grid});
  return grid;
}

hipError_t launch_validate(const SceneDev &sc, const float *qa, const float *qb, int64_t n_edges, float res,
                           const int32_t *n_states_opt, uint8_t *out_valid, const ValidateScratch &ws,
                           hipStream_t s, const std::pair<hipEvent_t, hipEvent_t> *ev_pair, uint64_t *totals,
                           int32_t *grid_out, int32_t *block_out) {
  const int64_t nb = scan_blocks(n_edges);
  const int64_t g256 = (n_edges + 255) / 256;
  if (g256 > 0x7fffffff || nb > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(count_states_kernel, dim3((unsigned)g256), dim3(256), 0, s, qa, qb, n_edges, sc.dof, res,
                     n_states_opt, ws.n_states, ws.flags);
  hipLaunchKernelGGL(scan_partials_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, s, ws.n_states, n_edges,
                     ws.block_sums);
  hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(kScanThreads), 0, s, ws.block_sums, nb, ws.counters);
  hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, s, ws.n_states, n_edges,
                     ws.block_sums, ws.offsets, ws.tile_first);
  const bool staged = use_staged(sc);
  const size_t lds = centre_lds_bytes(sc.n_robots) + (staged ? staged_floats(sc) * sizeof(float) : 0);
  const int grid = staged ? persistent_grid<true>(sc.n_robots, lds) : persistent_grid<false>(sc.n_robots, lds);
  if (grid_out) *grid_out = grid;
  if (block_out) *block_out = kWave * block_waves(sc.n_robots);
  if (ev_pair) (void)hipEventRecord(ev_pair->first, s);
  if (staged)
    hipLaunchKernelGGL(validate_tiles_kernel<true>, dim3(grid), dim3(kWave * block_waves(sc.n_robots)), lds, s, sc,
                       qa, qb, n_edges, ws.offsets, ws.tile_first, ws.flags, ws.counters, ws.partials);
  else
    hipLaunchKernelGGL(validate_tiles_kernel<false>, dim3(grid), dim3(kWave * block_waves(sc.n_robots)), lds, s, sc,
                       qa, qb, n_edges, ws.offsets, ws.tile_first, ws.flags, ws.counters, ws.partials);
  if (ev_pair) (void)hipEventRecord(ev_pair->second, s);
  hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)g256), dim3(256), 0, s, ws.flags, n_edges, out_valid,
                     ws.counters, ws.partials, grid, totals);
  return hipGetLastError();
}

}  // namespace mrpop
