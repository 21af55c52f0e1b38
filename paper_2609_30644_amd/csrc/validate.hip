// Composite edge validation: state counts, prefix scan, and the tile kernel.
//
// An edge (q_a, q_b) is checked at n discretised states (paper, Sec.
// "Multi-Thread Reassignment for Collision Checking").  The states of all
// edges form one global list (exclusive prefix sum of the per-edge counts);
// persistent workgroups take tiles of 64 consecutive list positions in a
// static grid-stride order.
//
// Mapping: one lane per state; a workgroup of W waves (up to 16) works on
// one tile at a time, and every arm's data is wave-uniform (scalar loads or
// LDS broadcasts) while consecutive states of an edge sit in neighbouring
// lanes and take the same branches.
//   1. Chains: the arms' link frames (modified DH) are composed in registers;
//      every link's coarse centre and (when they fit) the joints' sines and
//      cosines are published in LDS.
//   2. Environment jobs (arm, link), claimed from an LDS counter, largest
//      links first (or, without the cached sines and cosines, a static split
//      of every arm's links over S waves): the coarse sphere against every
//      obstacle (environment spheres and the bounding spheres of boxes) in
//      expanded form -- three FMAs from |c|^2 and a compare against a
//      per-(link, obstacle) row, four obstacles per step, compare masks in
//      scalar registers; flagged (lane, obstacle) pairs go to a per-wave LDS
//      queue and are tested one pair per lane (exact link-box distance for
//      boxes, then the link's fine spheres), so that the rare flagged pairs
//      do not make the whole wave wait on a few lanes.
//   3. After a barrier, the arm pairs that can reach each other are split
//      over the waves as (pair, link of the first arm) items: coarse
//      link-link tests from the LDS centres for the link pairs the pair's
//      static mask allows, and for flagged link pairs the two frames are
//      rebuilt and the fine spheres tested.
// A collision marks the edge in a flag word and marks all of the edge's lanes
// of the tile in an LDS mask, which the other waves read as they go.  In the
// plain order tiles do not read the flag words: the tiles of one edge run at
// the same time on different workgroups, so the check almost never skipped a
// state, and the coherent load it needs cost a memory round trip per tile.
// One-launch batches of more tiles than workgroups use a two-pass order
// instead (every K-th state of each edge first, see map_lanes_split), whose
// second-pass tiles do read them and skip the states of marked edges.
#include <hip/hip_ext.h>
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "device_common.h"

namespace mrpop {

constexpr int kScanThreads = 1024;
constexpr int kScanItems = 4;
constexpr int kScanChunk = kScanThreads * kScanItems;

enum : uint32_t { kFlagHit = 1u, kFlagNonFinite = 2u, kFlagTooLong = 4u };

// Batches of at most this many edges count as small for the tile shape.
constexpr int64_t kSmallBatchEdges = 1024;

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

// State count of edge e and its flag word (non-finite input, too long).
__device__ __forceinline__ int32_t edge_states(const float *__restrict__ qa, const float *__restrict__ qb, int64_t e,
                                               int dof, float res, const int32_t *__restrict__ n_opt, uint32_t *flag) {
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
  } else {
    const int32_t c = state_count_code(linf, true, res);
    if (c == kCodeTooLong) f = kFlagTooLong;
    else n = c;
  }
  *flag = f;
  return n;
}

__global__ __launch_bounds__(256) void count_states_kernel(const float *__restrict__ qa, const float *__restrict__ qb,
                                                           int64_t n_edges, int dof, float res,
                                                           const int32_t *__restrict__ n_opt,
                                                           int32_t *__restrict__ n_out, uint32_t *__restrict__ flags) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_edges) return;
  uint32_t f;
  n_out[e] = edge_states(qa, qb, e, dof, res, n_opt, &f);
  flags[e] = f;
}

// ---------------------------------------------------------------------------
// 2. exclusive prefix sum of the counts (three passes)
// ---------------------------------------------------------------------------

// One DPP move of a 64-bit value (both halves): lane i takes the value the
// control selects (0 where the source lies outside its row), in the rows of
// ROWS; the other rows take 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint64_t dpp64(uint64_t x) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)x, CTRL, ROWS, 0xf, true);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(x >> 32), CTRL, ROWS, 0xf, true);
  return ((uint64_t)hi << 32) | lo;
}

// Sum of v over the wave, in every lane, without LDS: an inclusive scan
// within each row of 16 lanes (row_shr 1, 2, 4, 8), then the rows' totals
// carried by row_bcast:15 (into rows 1 and 3) and row_bcast:31 (into rows 2
// and 3), so that lane 63 holds the sum; it is then read out uniformly.
// Every lane of the wave must be active.
__device__ __forceinline__ uint64_t wave_sum(uint64_t x) {
  x += dpp64<0x111, 0xf>(x);
  x += dpp64<0x112, 0xf>(x);
  x += dpp64<0x114, 0xf>(x);
  x += dpp64<0x118, 0xf>(x);
  x += dpp64<0x142, 0xa>(x);
  x += dpp64<0x143, 0xc>(x);
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)x, kWave - 1);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(x >> 32), kWave - 1);
  return ((uint64_t)hi << 32) | lo;
}

// Inclusive prefix sum over the wave, without LDS (every lane active): the
// row shifts of wave_sum, then each row's carry from the rows below, taken
// by row broadcasts with every row enabled and kept only in the rows that
// receive it (lane-index selects).
__device__ __forceinline__ uint64_t wave_inclusive_scan(uint64_t x, int lane) {
  x += dpp64<0x111, 0xf>(x);
  x += dpp64<0x112, 0xf>(x);
  x += dpp64<0x114, 0xf>(x);
  x += dpp64<0x118, 0xf>(x);
  const int row = lane >> 4;
  const uint64_t b15 = dpp64<0x142, 0xf>(x);  // lane 15 of the row below
  x += (row & 1) ? b15 : 0ull;                // rows 1 and 3
  const uint64_t b31 = dpp64<0x143, 0xf>(x);  // lane 31
  x += row >= 2 ? b31 : 0ull;                 // rows 2 and 3
  return x;
}

// Exclusive scan of one value per thread across the block; returns the
// exclusive prefix and writes the block total.
__device__ int64_t block_exclusive_scan(int64_t v, int64_t *total) {
  __shared__ int64_t wave_sums[kScanThreads / kWave];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int64_t x = (int64_t)wave_inclusive_scan((uint64_t)v, lane);
  if (lane == kWave - 1) wave_sums[wid] = x;
  __syncthreads();
  if (wid == 0) {
    const int nw = blockDim.x / kWave;
    const int64_t w = (int64_t)wave_inclusive_scan(lane < nw ? (uint64_t)wave_sums[lane] : 0ull, lane);
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
      if (tile_first)
        for (int64_t tl = (run + kWave - 1) / kWave; tl * kWave < run + v[i] && tl < kTileFirstCap; ++tl)
          tile_first[tl] = (int32_t)(base + i);
    }
    run += v[i];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) offsets[n_edges] = block_sums[gridDim.x];
}

// Small batches (small_scan): counts, flags, exclusive offsets, the tile
// table and the totals in one workgroup, kScanThreads edges at a time (one
// launch instead of four).
__global__ __launch_bounds__(kScanThreads) void count_scan_small_kernel(
    const float *__restrict__ qa, const float *__restrict__ qb, int64_t n_edges, int dof, float res,
    const int32_t *__restrict__ n_opt, int32_t *__restrict__ n_out, uint32_t *__restrict__ flags,
    int64_t *__restrict__ offsets, int32_t *__restrict__ tile_first, uint64_t *__restrict__ counters) {
  int64_t carry = 0;
  for (int64_t e0 = 0; e0 < n_edges; e0 += kScanThreads) {
    const int64_t e = e0 + threadIdx.x;
    int64_t v = 0;
    if (e < n_edges) {
      uint32_t f;
      v = edge_states(qa, qb, e, dof, res, n_opt, &f);
      n_out[e] = (int32_t)v;
      flags[e] = f;
    }
    int64_t total;
    const int64_t run = carry + block_exclusive_scan(v, &total);
    if (e < n_edges) {
      offsets[e] = run;
      for (int64_t tl = (run + kWave - 1) / kWave; tl * kWave < run + v && tl < kTileFirstCap; ++tl)
        tile_first[tl] = (int32_t)e;
    }
    carry += total;
  }
  if (threadIdx.x == 0) {
    offsets[n_edges] = carry;
    counters[0] = 0;
    counters[1] = (uint64_t)carry;
    for (int c = 2; c < 16; ++c) counters[c] = 0;
  }
}

// Many-scene batches of at most kSegSmallMax segments whose edges pass
// small_scan (at the largest dof): one workgroup does the work of seg_count, the scan, seg_tiles and
// seg_table, from segments passed by value, which it also stores to
// segs_out for the tile and final kernels.  Every thread revisits only the
// edges it wrote itself.
struct SegSmall {
  ValSeg s[kSegSmallMax];
};
static_assert(sizeof(SegSmall) + 128 <= 4096, "segment table exceeds the kernel argument space");

__global__ __launch_bounds__(kScanThreads) void seg_prep_small_kernel(
    SegSmall in, int n_segs, int64_t n_flat, ValSeg *__restrict__ segs_out, int32_t *__restrict__ n_states,
    uint32_t *__restrict__ flags, int32_t *__restrict__ edge_seg, int64_t *__restrict__ off,
    int32_t *__restrict__ tile_first, int32_t *__restrict__ tile_seg, uint64_t *__restrict__ batch) {
  __shared__ int64_t s_start[kSegSmallMax], s_tile0[kSegSmallMax];
  if (threadIdx.x < kSegSmallMax) s_start[threadIdx.x] = -1;
  __syncthreads();
  int64_t carry = 0;
  for (int64_t f0 = 0; f0 < n_flat; f0 += kScanThreads) {
    const int64_t f = f0 + threadIdx.x;
    int64_t v = 0;
    int k = 0;
    if (f < n_flat) {
      while (k + 1 < n_segs && f >= in.s[k + 1].edge0) ++k;
      const ValSeg &g = in.s[k];
      uint32_t fl;
      v = edge_states(g.qa, g.qb, f - g.edge0, g.sc.dof, g.res, nullptr, &fl);
      n_states[f] = (int32_t)v;
      flags[f] = fl;
      edge_seg[f] = k;
    }
    int64_t total;
    const int64_t run = carry + block_exclusive_scan(v, &total);
    if (f < n_flat) {
      off[f] = run;
      if (f == in.s[k].edge0) s_start[k] = run;
    }
    carry += total;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    off[n_flat] = carry;
    for (int k = n_segs - 1; k >= 0; --k)  // empty segments start where the next one does
      if (s_start[k] < 0) s_start[k] = k + 1 < n_segs ? s_start[k + 1] : carry;
    int64_t t = 0;
    for (int k = 0; k < n_segs; ++k) {
      const int64_t states = (k + 1 < n_segs ? s_start[k + 1] : carry) - s_start[k];
      ValSeg g = in.s[k];
      g.tile0 = t;
      s_tile0[k] = t;
      t += (states + kWave - 1) / kWave;
      segs_out[k] = g;
      for (int i = 0; i < 16; ++i) g.counters[i] = 0;
      g.counters[1] = (uint64_t)states;
    }
    batch[0] = 0;
    batch[1] = (uint64_t)t;
    batch[2] = t > kTileFirstCap ? 1 : 0;
    for (int c = 3; c < 16; ++c) batch[c] = 0;
  }
  __syncthreads();
  for (int64_t f0 = 0; f0 < n_flat; f0 += kScanThreads) {
    const int64_t f = f0 + threadIdx.x;
    if (f >= n_flat) continue;
    const int k = edge_seg[f];
    const int64_t run = off[f] - s_start[k], v = n_states[f];
    for (int64_t tl = (run + kWave - 1) / kWave; tl * kWave < run + v; ++tl) {
      const int64_t t = s_tile0[k] + tl;
      if (t >= kTileFirstCap) break;
      tile_first[t] = (int32_t)f;
      tile_seg[t] = k;
    }
  }
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

__device__ __forceinline__ int64_t find_edge(const int32_t *__restrict__ off, int64_t n_edges, int64_t s) {
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

// Per-wave LDS of the environment stage: the current link's frame at every
// lane's state (12 floats x 64, one row per element) and the queue of flagged
// (lane, obstacle) pairs awaiting the fine test.
constexpr int kGroup = 4;                           // obstacles per coarse step
constexpr int kQueueFlushAt = kWave;                 // flush once more items than this are queued
constexpr int kQueueCap = kQueueFlushAt + kGroup * kWave;
constexpr int kWaveLdsFloats = 12 * kWave + kQueueCap;
static_assert(kClusterSize == 2 * kGroup, "a cluster's rows are two groups");

// Scene data the tile kernel reads at lane-varying indices inside its loops:
// obstacle spheres and boxes, fine spheres, link ranges and coarse radii.
// STAGED: copied to LDS once per persistent workgroup.  Otherwise: the scene
// arrays themselves.  (The coarse filter rows, the same for every lane,
// always come through the scalar cache: from LDS each read would write them
// into every lane's registers, which costs more LDS bandwidth than the tests
// they feed.)
template <bool STAGED>
struct Src;

template <>
struct Src<true> {
  const float4 *env_s;   // [Ns]
  const float4 *boxes;   // [Nb][2]
  const float4 *fine;    // [M][sph_stride]
  const int32_t *lstart; // [M][kMaxLinks + 1]
  const float *crad;     // [M][kMaxLinks]
  int ns, nb, stride;
  __device__ float4 sphere(int k) const { return env_s[k]; }
  __device__ float4 box(int i) const { return boxes[i]; }
  __device__ float4 sph(int m, int i) const { return fine[m * stride + i]; }
  __device__ int ls(int m, int l) const { return lstart[m * (kMaxLinks + 1) + l]; }
  __device__ float rad(int m, int l) const { return crad[m * kMaxLinks + l]; }
};

template <>
struct Src<false> {
  cptr<float4> fine, coarse;
  const float4 *env_s, *boxes;  // read at lane-varying indices
  cptr<int32_t> lstart;
  int ns, nb, stride;
  __device__ float4 sphere(int k) const { return env_s[k]; }
  __device__ float4 box(int i) const { return boxes[i]; }
  __device__ float4 sph(int m, int i) const { return ld4(fine, (int64_t)m * stride + i); }
  __device__ int ls(int m, int l) const { return lstart[m * (kMaxLinks + 1) + l]; }
  __device__ float rad(int m, int l) const { return ld4(coarse, m * kMaxLinks + l).w; }
};

// LDS floats needed to stage a scene.
__host__ __device__ inline size_t staged_floats(const SceneDev &sc) {
  const size_t M = sc.n_models;
  return (size_t)sc.n_env_spheres * 4 + (size_t)sc.n_env_boxes * 8 + M * (size_t)sc.sph_stride * 4 +
         M * (kMaxLinks + 1) + M * kMaxLinks;
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
  float4 *p = (float4 *)stage;
  s.env_s = p;
  for (int i = threadIdx.x; i < s.ns; i += blockDim.x) p[i] = sc.env_s[i];
  p += s.ns;
  s.boxes = p;
  for (int i = threadIdx.x; i < 2 * s.nb; i += blockDim.x) p[i] = sc.env_b[i];
  p += 2 * s.nb;
  s.fine = p;
  for (int i = threadIdx.x; i < M * s.stride; i += blockDim.x) p[i] = sc.fine[i];
  p += M * s.stride;
  int32_t *ip = (int32_t *)p;
  s.lstart = ip;
  for (int i = threadIdx.x; i < M * (kMaxLinks + 1); i += blockDim.x) ip[i] = sc.link_start[i];
  float *fp = (float *)(ip + M * (kMaxLinks + 1));
  s.crad = fp;
  for (int i = threadIdx.x; i < M * kMaxLinks; i += blockDim.x) fp[i] = sc.coarse[i].w;
  __syncthreads();
  return s;
}

template <>
__device__ Src<false> make_src<false>(const SceneDev &sc, float *) {
  Src<false> s;
  s.env_s = sc.env_s;
  s.boxes = sc.env_b;
  s.fine = as_const(sc.fine);
  s.coarse = as_const(sc.coarse);
  s.lstart = as_const(sc.link_start);
  s.ns = sc.n_env_spheres;
  s.nb = sc.n_env_boxes;
  s.stride = sc.sph_stride;
  return s;
}

// Orders this wave's LDS accesses made by different lanes (LDS operations of
// one wave are performed in order; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Fine test of the queued (lane, obstacle) pairs of link l, one pair per
// lane: the frame of the pair's state comes from LDS; an environment sphere
// is tested against every fine sphere of the link, a box first against the
// link's coarse sphere (exact distance), then against the fine spheres.  A
// collision sets the state's bit in *hitw.
template <bool STAGED>
__device__ void flush_queue(const Src<STAGED> &src, int m, int l, float4 cs, const float *fr,
                            const uint32_t *queue, int qn, unsigned long long *hitw, int lane, WorkCount &wc) {
  wave_lds_sync();
  const int x0 = src.ls(m, l), x1 = src.ls(m, l + 1);
  // with fewer items than lanes, each item gets a group of L lanes that share
  // its sphere loop (L a power of two, wave-uniform)
  int L = 1;
  while (L < kWave && qn * (2 * L) <= kWave) L *= 2;
  const int sub = lane & (L - 1);
  for (int i0 = 0; i0 < qn; i0 += kWave / L) {
    const int i = i0 + lane / L;
    if (i >= qn) continue;
    const uint32_t item = queue[i];
    const int s = (int)(item & (kWave - 1));
    const int k = (int)(item >> 6);
    Frame G;
    G.r00 = fr[0 * kWave + s]; G.r01 = fr[1 * kWave + s]; G.r02 = fr[2 * kWave + s]; G.t0 = fr[3 * kWave + s];
    G.r10 = fr[4 * kWave + s]; G.r11 = fr[5 * kWave + s]; G.r12 = fr[6 * kWave + s]; G.t1 = fr[7 * kWave + s];
    G.r20 = fr[8 * kWave + s]; G.r21 = fr[9 * kWave + s]; G.r22 = fr[10 * kWave + s]; G.t2 = fr[11 * kWave + s];
    bool h = false;
    if (k < src.ns) {
      const float4 o = src.sphere(k);
      for (int x = x0 + sub; x < x1; x += L) {
        const float4 p = src.sph(m, x);
        const float3 w = apply(G, p.x, p.y, p.z);
        const float rr = p.w + o.w;
        ++wc.fine_s;
        if (dist2(w, o) < rr * rr) {
          h = true;
          break;
        }
      }
    } else {
      const int kb = k - src.ns;
      const float4 lo = src.box(2 * kb), hi = src.box(2 * kb + 1);
      const float3 c = apply(G, cs.x, cs.y, cs.z);
      if (sub == 0) ++wc.box_exact;  // (every lane of the group makes the same test)
      if (box_dist2(c, lo, hi) < cs.w * cs.w) {
        for (int x = x0 + sub; x < x1; x += L) {
          const float4 p = src.sph(m, x);
          const float3 w = apply(G, p.x, p.y, p.z);
          ++wc.fine_b;
          if (box_dist2(w, lo, hi) < p.w * p.w) {
            h = true;
            break;
          }
        }
      }
    }
    if (h) atomicOr(hitw, 1ull << s);
  }
  wave_lds_sync();
}

// Environment tests of link l of arm r (model m) at every lane's state, given
// the link's frame F and its coarse centre c (both at the lane's own state):
// the frame goes to the wave's LDS slot, the coarse sphere is tested against
// the obstacles of the link's list (those within its reach of the arm's
// base) in expanded form (three FMAs and a compare), flagged (lane,
// obstacle) pairs are queued and get their fine tests one pair per lane.
// Returns the lanes whose state collides; their edges are marked in *dead.
template <bool STAGED>
__device__ bool link_env(const SceneDev &sc, const Src<STAGED> &src, int r, int m, int l, const Frame &F, float3 c,
                         bool live, uint64_t emask, float *fr, uint32_t *queue, unsigned long long *hitw,
                         unsigned long long *dead, int lane, WorkCount &wc) {
  const float4 cs = ld4(as_const(sc.coarse), m * kMaxLinks + l);
  if (cs.w < 0.f) return false;  // a link without spheres
  // the link's list: row offset, rows (padded), obstacles, cluster-row
  // offset, cluster rows (padded), clusters
  const cptr<int32_t> meta = as_const(sc.link_lists) + (r * kMaxLinks + l) * 8;
  const int row0 = meta[0], n8 = meta[1], N = meta[2], crow0 = meta[3], nc8 = meta[4], nc = meta[5];
  if (live) {
    ++wc.links;
    wc.env_tests += nc > 0 ? nc : N;  // (with clusters, member rows are counted as they are tested)
  }
  if (N == 0) return false;
  const float c2 = fmaf(c.z, c.z, fmaf(c.y, c.y, c.x * c.x));
  if (lane == 0) *hitw = 0ull;
  fr[0 * kWave + lane] = F.r00; fr[1 * kWave + lane] = F.r01; fr[2 * kWave + lane] = F.r02;
  fr[3 * kWave + lane] = F.t0;  fr[4 * kWave + lane] = F.r10; fr[5 * kWave + lane] = F.r11;
  fr[6 * kWave + lane] = F.r12; fr[7 * kWave + lane] = F.t1;  fr[8 * kWave + lane] = F.r20;
  fr[9 * kWave + lane] = F.r21; fr[10 * kWave + lane] = F.r22; fr[11 * kWave + lane] = F.t2;
  const float4 csr = make_float4(cs.x, cs.y, cs.z, src.rad(m, l));
  const uint64_t livem = __builtin_amdgcn_ballot_w64(live);
  const cptr<int32_t> obs = as_const(sc.row_obs) + row0;
  int qn = 0;  // wave-uniform queue length
  // one group of kGroup rows (k0 onwards in the list): the coarse tests, and
  // the flagged pairs queued with the row's obstacle (flushed once the queue
  // is long enough)
  auto group_tests = [&](const float4 (&rw)[kGroup], int k0) {
    bool h[kGroup];
    uint64_t b[kGroup], any = 0;
#pragma unroll
    for (int i = 0; i < kGroup; ++i) {
      const float t = fmaf(c.z, rw[i].z, fmaf(c.y, rw[i].y, fmaf(c.x, rw[i].x, c2)));
      h[i] = t < -rw[i].w;
      b[i] = __builtin_amdgcn_ballot_w64(h[i]);
      any |= b[i];
    }
    if ((any & livem) == 0ull) return;
#pragma unroll
    for (int i = 0; i < kGroup; ++i) {
      const uint64_t bi = b[i] & livem;
      if (bi == 0ull) continue;
      if (h[i] && live)
        queue[qn + __builtin_amdgcn_mbcnt_hi((uint32_t)(bi >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bi, 0u))] =
            (uint32_t)lane | ((uint32_t)obs[k0 + i] << 6);
      qn += __popcll(bi);
    }
    if (qn > kQueueFlushAt) {
      flush_queue<STAGED>(src, m, l, csr, fr, queue, qn, hitw, lane, wc);
      qn = 0;
    }
  };
  // Two groups per step over two row buffers, software-pipelined: each
  // group's scalar load is in flight while the group before it is tested.
  // n8 is a multiple of 2 kGroup; the last step's prefetch reads the group
  // that follows the list's rows (the next list's, or the padding after the
  // last list) and leaves it unused.
  auto load = [](cptr<float> p, float4 (&r)[kGroup]) {
#pragma unroll
    for (int i = 0; i < kGroup; ++i) r[i] = make_float4(p[4 * i], p[4 * i + 1], p[4 * i + 2], p[4 * i + 3]);
  };
  cptr<float> p = (cptr<float>)(as_const(sc.rows) + row0);
  float4 ra[kGroup], rb[kGroup];
  if (nc == 0) {
    load(p, ra);
    for (int k0 = 0; k0 < n8; k0 += 2 * kGroup) {
      load(p + 4 * (k0 + kGroup), rb);
      __builtin_amdgcn_sched_barrier(0);  // keep each load ahead of the tests it overlaps
      group_tests(ra, k0);
      load(p + 4 * (k0 + 2 * kGroup), ra);
      __builtin_amdgcn_sched_barrier(0);
      group_tests(rb, k0 + kGroup);
    }
  } else {
    // Clusters in chunks of 64: first the chunk's cluster rows, in the same
    // pipelined pairs of groups, into a mask of the clusters that pass for a
    // live lane; then the member rows of those clusters (two groups of kGroup
    // each), again with each group's load issued before the group ahead of
    // it is tested.
    auto cluster_mask = [&](const float4 (&cw)[kGroup], int i0, uint64_t &pm) {
#pragma unroll
      for (int i = 0; i < kGroup; ++i) {
        const float t = fmaf(c.z, cw[i].z, fmaf(c.y, cw[i].y, fmaf(c.x, cw[i].x, c2)));
        if (__builtin_amdgcn_ballot_w64(t < -cw[i].w) & livem) pm |= 1ull << (i0 + i);
      }
    };
    cptr<float> pc = (cptr<float>)(as_const(sc.crows) + crow0);
    for (int ch = 0; ch < nc8; ch += 64) {
      const int n_ch = min(64, nc8 - ch);  // a multiple of 2 kGroup
      uint64_t pm = 0;
      load(pc, ra);
      for (int i0 = 0; i0 < n_ch; i0 += 2 * kGroup) {
        load(pc + 4 * kGroup, rb);
        __builtin_amdgcn_sched_barrier(0);
        cluster_mask(ra, i0, pm);
        load(pc + 8 * kGroup, ra);
        __builtin_amdgcn_sched_barrier(0);
        cluster_mask(rb, i0 + kGroup, pm);
        pc += 8 * kGroup;
      }
      if (pm == 0ull) continue;
      int k0 = (ch + __builtin_ctzll(pm)) * kClusterSize;
      pm &= pm - 1;
      load(p + 4 * k0, ra);
      for (;;) {
        if (live) wc.env_tests += min(kClusterSize, N - k0);
        load(p + 4 * (k0 + kGroup), rb);
        __builtin_amdgcn_sched_barrier(0);
        group_tests(ra, k0);
        const int k1 = pm ? (ch + __builtin_ctzll(pm)) * kClusterSize : -1;
        if (k1 >= 0) load(p + 4 * k1, ra);
        __builtin_amdgcn_sched_barrier(0);
        group_tests(rb, k0 + kGroup);
        if (k1 < 0) break;
        pm &= pm - 1;
        k0 = k1;
      }
    }
  }
  if (qn > 0) flush_queue<STAGED>(src, m, l, csr, fr, queue, qn, hitw, lane, wc);
  const bool hit = live && ((*hitw >> lane) & 1ull);
  if (hit) atomicOr(dead, (unsigned long long)emask);
  return hit;
}

// Kinematic chain of arm r (model m) at every lane's state: every link's
// frame in turn (modified DH), its coarse centre published in LDS for the
// later stages, and with sc_lds the joints' sines and cosines cached there.
// visit(l, F, c) runs at each link.
template <class Visit>
__device__ void arm_chain(const SceneDev &sc, int r, int m, const float (&qv)[kMaxJoints], float *cen, float *sc_lds,
                          int lane, Visit &&visit) {
  const int nj = as_const(sc.nj)[m];
  Frame F = base_frame(sc, r);
  for (int l = 0; l <= nj; ++l) {
    if (l > 0) {
      float sn, cs;
      sincosf(qv[l - 1] + as_const(sc.theta_off)[m * kMaxJoints + l - 1], &sn, &cs);
      joint_step_sc(F, ld4(as_const(sc.dh), m * kMaxJoints + l - 1), sn, cs);
      if (sc_lds) {
        float *q = sc_lds + ((r * kMaxJoints + l - 1) * 2) * kWave + lane;
        q[0] = sn;
        q[kWave] = cs;
      }
    }
    const float4 co = ld4(as_const(sc.coarse), m * kMaxLinks + l);
    const float3 c = apply(F, co.x, co.y, co.z);
    float *slot = cen + ((r * kMaxLinks + l) * 3) * kWave + lane;
    slot[0] = c.x;
    slot[kWave] = c.y;
    slot[2 * kWave] = c.z;
    if (!visit(l, F, c)) break;
  }
}

// Environment stage of arm r (model m) for the links l with l % S == part
// (static split: every wave of the arm runs the whole chain and tests its own
// links).  Returns true for lanes whose state collides.
template <bool STAGED>
__device__ bool arm_env(const SceneDev &sc, const Src<STAGED> &src, int r, int m, int part, int S,
                        const float (&qv)[kMaxJoints], bool live, uint64_t emask, float *cen, float *sc_lds,
                        float *fr, uint32_t *queue, unsigned long long *hitw, unsigned long long *dead, int lane,
                        WorkCount &wc) {
  bool hit = false;
  if (live && part == 0) ++wc.chains;
  arm_chain(sc, r, m, qv, cen, sc_lds, lane, [&](int l, const Frame &F, float3 c) {
    if (l % S != part) return true;  // another wave tests this link
    live = live && !((dead_mask(dead) >> lane) & 1ull);
    if (__ballot(live) == 0ull) return false;  // nothing left to test in this wave
    if (link_env<STAGED>(sc, src, r, m, l, F, c, live, emask, fr, queue, hitw, dead, lane, wc)) {
      hit = true;
      live = false;
    }
    return true;
  });
  return hit;
}

// Frame of link `link` of arm r (model m) at the state of lane s, composed
// from the sines and cosines the environment stage cached in LDS (the same
// operations as the environment stage's chain, so the same frame).  Arm,
// model and link may differ between lanes.
__device__ Frame frame_cached(const SceneDev &sc, int r, int m, int link, int s, const float *sc_lds) {
  const float *p = sc.base + 12 * r;
  Frame F;
  F.r00 = p[0]; F.r01 = p[1]; F.r02 = p[2]; F.t0 = p[3];
  F.r10 = p[4]; F.r11 = p[5]; F.r12 = p[6]; F.t1 = p[7];
  F.r20 = p[8]; F.r21 = p[9]; F.r22 = p[10]; F.t2 = p[11];
  for (int j = 1; j <= link; ++j) {
    const float *q = sc_lds + ((r * kMaxJoints + j - 1) * 2) * kWave + s;
    joint_step_sc(F, sc.dh[m * kMaxJoints + j - 1], q[0], q[kWave]);
  }
  return F;
}

// Fine test of queued arm-pair items (lane s, pair p, link a of the pair's
// first arm, link b of its second), one item per lane: both frames come from
// the cached sines and cosines; spheres of link b that miss link a's coarse
// sphere cannot touch any sphere of link a and are dropped first (the coarse
// sphere contains every fine sphere of its link), then the remaining sphere
// pairs are tested.  A collision sets the state's bit in *hitw.
// Without the cache (scenes with many arms, where it does not fit in LDS):
// the same frame rebuilt from the joint values of the state that lane s
// holds (ls: that lane's state, fetched by the caller).
__device__ Frame frame_rebuilt(const SceneDev &sc, int r, int m, int link, const LaneState &ls) {
  const float *p = sc.base + 12 * r;
  Frame F;
  F.r00 = p[0]; F.r01 = p[1]; F.r02 = p[2]; F.t0 = p[3];
  F.r10 = p[4]; F.r11 = p[5]; F.r12 = p[6]; F.t1 = p[7];
  F.r20 = p[8]; F.r21 = p[9]; F.r22 = p[10]; F.t2 = p[11];
  const int q0 = sc.q_off[r];
  for (int j = 1; j <= link; ++j) {
    float sn, cs;
    sincosf(joint_value(ls, q0 + j - 1) + sc.theta_off[m * kMaxJoints + j - 1], &sn, &cs);
    joint_step_sc(F, sc.dh[m * kMaxJoints + j - 1], sn, cs);
  }
  return F;
}

// LaneState of lane s (every lane of the wave must take part).
__device__ __forceinline__ LaneState lane_state_of(const LaneState &st, int s) {
  LaneState o;
  const uint64_t a = (uint64_t)st.qa, b = (uint64_t)st.qb;
  o.qa = (const float *)(((uint64_t)(uint32_t)__shfl((int)(a >> 32), s, kWave) << 32) |
                         (uint32_t)__shfl((int)(uint32_t)a, s, kWave));
  o.qb = (const float *)(((uint64_t)(uint32_t)__shfl((int)(b >> 32), s, kWave) << 32) |
                         (uint32_t)__shfl((int)(uint32_t)b, s, kWave));
  o.t = __shfl(st.t, s, kWave);
  o.last = __shfl((int)st.last, s, kWave) != 0;
  return o;
}

template <bool STAGED, bool CACHE>
__device__ void flush_pairs(const SceneDev &sc, const Src<STAGED> &src, const float *cen, const float *sc_lds,
                            const LaneState &st, const uint32_t *queue, int qn, unsigned long long *hitw, int lane,
                            WorkCount &wc) {
  wave_lds_sync();
  // with fewer items than lanes, each item gets a group of L lanes that share
  // its sphere loop (L a power of two, wave-uniform)
  int L = 1;
  while (L < kWave && qn * (2 * L) <= kWave) L *= 2;
  const int sub = lane & (L - 1);
  for (int i0 = 0; i0 < qn; i0 += kWave / L) {
    const int i = i0 + lane / L;
    const uint32_t item = i < qn ? queue[i] : 0u;
    const int s = (int)(item & (kWave - 1)), a = (int)((item >> 6) & 7u), b = (int)((item >> 9) & 7u);
    const int p = (int)(item >> 12);
    const LaneState ls = CACHE ? st : lane_state_of(st, s);  // all lanes active here
    if (i >= qn) continue;
    const int ai = sc.pairs[2 * p], aj = sc.pairs[2 * p + 1];
    const int mi = sc.model[ai], mj = sc.model[aj];
    const float *pa = cen + ((ai * kMaxLinks + a) * 3) * kWave + s;
    const float *pb = cen + ((aj * kMaxLinks + b) * 3) * kWave + s;
    const float4 ca = make_float4(pa[0], pa[kWave], pa[2 * kWave], src.rad(mi, a));
    const float4 cb = make_float4(pb[0], pb[kWave], pb[2 * kWave], src.rad(mj, b));
    const Frame Fa = CACHE ? frame_cached(sc, ai, mi, a, s, sc_lds) : frame_rebuilt(sc, ai, mi, a, ls);
    const Frame Fb = CACHE ? frame_cached(sc, aj, mj, b, s, sc_lds) : frame_rebuilt(sc, aj, mj, b, ls);
    const int x0 = src.ls(mi, a), x1 = src.ls(mi, a + 1), y0 = src.ls(mj, b), y1 = src.ls(mj, b + 1);
    // spheres of link b within reach of link a's coarse sphere (links with
    // more than 64 spheres keep the rest unfiltered)
    const int ny = y1 - y0 < 64 ? y1 - y0 : 64;
    uint64_t ym = 0;
    for (int y = y0; y < y0 + ny; ++y) {
      const float4 q = src.sph(mj, y);
      const float3 wy = apply(Fb, q.x, q.y, q.z);
      const float rr = q.w + ca.w;
      if (sub == 0) ++wc.fine_rr;  // (every lane of the group computes the same mask)
      if (dist2(wy, ca) < rr * rr) ym |= 1ull << (y - y0);
    }
    const bool rest = y1 - y0 > 64;
    bool h = false;
    for (int x = x0 + sub; x < x1 && (ym != 0ull || rest) && !h; x += L) {
      const float4 q = src.sph(mi, x);
      const float3 wx = apply(Fa, q.x, q.y, q.z);
      const float rx = q.w + cb.w;
      ++wc.fine_rr;
      if (!(dist2(wx, cb) < rx * rx)) continue;
      for (int y = y0; y < y1; ++y) {
        if (y - y0 < 64 && !((ym >> (y - y0)) & 1ull)) continue;
        const float4 t = src.sph(mj, y);
        const float3 wy = apply(Fb, t.x, t.y, t.z);
        const float rr = q.w + t.w;
        ++wc.fine_rr;
        if (dist2(wx, wy) < rr * rr) {
          h = true;
          break;
        }
      }
    }
    if (h) atomicOr(hitw, 1ull << s);
  }
  wave_lds_sync();
}

// Arm-pair stage of one wave: items (pair p, link a of the pair's first arm)
// p * kMaxLinks + a = w, w + W, ...; coarse link-link tests on the published
// centres for the link pairs the pair's static mask allows, flagged (lane,
// pair, a, b) items queued and tested by flush_pairs.  Returns true for lanes
// whose state collides.
template <bool STAGED, bool CACHE>
__device__ bool arm_pairs(const SceneDev &sc, const Src<STAGED> &src, const float *cen, const float *sc_lds, int w,
                          int W, bool live, const LaneState &st, uint64_t emask, uint32_t *queue,
                          unsigned long long *hitw, unsigned long long *dead, int lane, WorkCount &wc) {
  if (lane == 0) *hitw = 0ull;
  int qn = 0;
  for (int q = w; q < sc.n_pairs * kMaxLinks; q += W) {
    const int p = q / kMaxLinks, a = q - p * kMaxLinks;
    const uint32_t row = (uint32_t)(as_const(sc.pair_links)[p] >> (a * kMaxLinks)) & 0xffu;
    if (row == 0u) continue;
    live = live && !((dead_mask(dead) >> lane) & 1ull);
    const uint64_t livem = __builtin_amdgcn_ballot_w64(live);
    if (livem == 0ull) break;
    const int pi = as_const(sc.pairs)[2 * p], pj = as_const(sc.pairs)[2 * p + 1];
    const int mi = as_const(sc.model)[pi], mj = as_const(sc.model)[pj];
    const float ra = src.rad(mi, a);
    const float *pa = cen + ((pi * kMaxLinks + a) * 3) * kWave + lane;
    const float3 ca = make_float3(pa[0], pa[kWave], pa[2 * kWave]);
    for (int b = 0; b < kMaxLinks; ++b) {
      if (!((row >> b) & 1u)) continue;
      const float *pb = cen + ((pj * kMaxLinks + b) * 3) * kWave + lane;
      const float3 cb = make_float3(pb[0], pb[kWave], pb[2 * kWave]);
      const float rs = ra + src.rad(mj, b);
      if (live) ++wc.rr_coarse;
      const bool h = dist2(ca, cb) < rs * rs;
      const uint64_t bm = __builtin_amdgcn_ballot_w64(h) & livem;
      if (bm == 0ull) continue;
      if (h && live)
        queue[qn + __builtin_amdgcn_mbcnt_hi((uint32_t)(bm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bm, 0u))] =
            (uint32_t)lane | ((uint32_t)a << 6) | ((uint32_t)b << 9) | ((uint32_t)p << 12);
      qn += __popcll(bm);
      if (qn > kQueueFlushAt) {
        flush_pairs<STAGED, CACHE>(sc, src, cen, sc_lds, st, queue, qn, hitw, lane, wc);
        qn = 0;
      }
    }
  }
  if (qn > 0) flush_pairs<STAGED, CACHE>(sc, src, cen, sc_lds, st, queue, qn, hitw, lane, wc);
  const bool hit = live && ((*hitw >> lane) & 1ull);
  if (hit) atomicOr(dead, (unsigned long long)emask);
  return hit;
}

// LDS floats before the per-wave areas: published coarse centres
// [R][kMaxLinks][3][64] and cached joint sines/cosines [R][kMaxJoints][2][64].
__host__ __device__ inline size_t tile_shared_floats(int n_robots, int cache_sc) {
  return (size_t)n_robots * (kMaxLinks * 3 + (cache_sc ? kMaxJoints * 2 : 0)) * kWave;
}

// Lanes of one tile: lane i holds list position s0 + i (positions relative
// to `base`, the list offset of the first edge considered, e_base its index);
// my_off is off[e0 + lane] - base (clamped to the last edge).  Returns the
// lane's state, whether it is active, its edge and the lanes of the tile on
// the same edge.
struct TileLanes {
  LaneState st;
  bool act;
  int64_t e;
  uint64_t emask;
};

__device__ __forceinline__ TileLanes map_lanes(int64_t s0, int64_t total, int64_t e0, int64_t my_off,
                                               const int64_t *__restrict__ off, int64_t base, int64_t e_base,
                                               const float *qa, const float *qb, int dof, int lane) {
  TileLanes t;
  const int64_t s = s0 + lane;
  t.act = s < total;
  // the tile starts in edge e0 and spans at most 64 consecutive edges; a
  // binary search over lanes finds the last edge starting at or before the
  // lane's position
  int pos = 0;
#pragma unroll
  for (int step = kWave / 2; step > 0; step >>= 1) {
    const int cand = pos + step;
    const int64_t o = __shfl(my_off, cand, kWave);
    if (o <= s) pos = cand;
  }
  t.e = e0 + pos;
  const int64_t e_start = __shfl(my_off, pos, kWave);
  int64_t e_end = __shfl(my_off, pos < kWave - 1 ? pos + 1 : pos, kWave);
  if (t.act && pos == kWave - 1) e_end = off[t.e + 1] - base;  // active lanes are on a real edge
  t.st = LaneState{qa, qb, 0.f, false};
  t.emask = 0;
  if (t.act) {
    const int64_t n = e_end - e_start;
    const int64_t k = s - e_start;
    t.st.qa = qa + (t.e - e_base) * dof;
    t.st.qb = qb + (t.e - e_base) * dof;
    t.st.last = n > 1 && k == n - 1;
    t.st.t = n > 1 ? (float)k / (float)(n - 1) : 0.f;
    const int lo = (int)((e_start > s0 ? e_start : s0) - s0);
    const int hi = (int)((e_end < s0 + kWave ? e_end : s0 + kWave) - s0);
    t.emask = (hi - lo >= 64 ? ~0ull : ((1ull << (hi - lo)) - 1ull)) << lo;
  }
  return t;
}

// Two-pass state order of a small batch.  The list holds 2 E segments:
// segment e < E is the first pass of edge e, its states k = r0, r0 + K, ...,
// n - 1 (every K-th state counted back from q_b, r0 = (n - 1) mod K), and
// segment E + e the edge's other states in increasing order.  seg[] holds the
// segments' exclusive offsets (2 E + 1 entries).  Lane i holds list position
// s0 + i; the result names the real edge and state, so that the states are
// the same floats as in the plain order.
__device__ __forceinline__ TileLanes map_lanes_split(int64_t s0, int64_t total, int64_t g0, int64_t my_off,
                                                     const int32_t *seg, int n_edges, int K, const float *qa,
                                                     const float *qb, int dof, int lane) {
  TileLanes t;
  const int64_t s = s0 + lane;
  t.act = s < total;
  int pos = 0;
#pragma unroll
  for (int step = kWave / 2; step > 0; step >>= 1) {
    const int cand = pos + step;
    const int64_t o = __shfl(my_off, cand, kWave);
    if (o <= s) pos = cand;
  }
  const int64_t g = g0 + pos;
  const int64_t g_start = __shfl(my_off, pos, kWave);
  int64_t g_end = __shfl(my_off, pos < kWave - 1 ? pos + 1 : pos, kWave);
  if (t.act && pos == kWave - 1) g_end = seg[g + 1];
  const bool second = g >= n_edges;
  t.e = second ? g - n_edges : g;
  t.st = LaneState{qa, qb, 0.f, false};
  t.emask = 0;
  if (t.act) {
    const int64_t e = t.e;
    // (the whole list holds fewer than 2^31 states)
    const int n_other = second ? seg[e + 1] - seg[e] : seg[n_edges + e + 1] - seg[n_edges + e];
    const int n = (int)(g_end - g_start) + n_other;
    const int j = (int)(s - g_start);
    const int r0 = (n - 1) % K;
    const int k = !second ? r0 + j * K : (j < r0 ? j : r0 + 1 + ((j - r0) / (K - 1)) * K + (j - r0) % (K - 1));
    t.st.qa = qa + e * dof;
    t.st.qb = qb + e * dof;
    t.st.last = n > 1 && k == n - 1;
    t.st.t = n > 1 ? (float)k / (float)(n - 1) : 0.f;
    const int lo = (int)((g_start > s0 ? g_start : s0) - s0);
    const int hi = (int)((g_end < s0 + kWave ? g_end : s0 + kWave) - s0);
    t.emask = (hi - lo >= 64 ? ~0ull : ((1ull << (hi - lo)) - 1ull)) << lo;
  }
  return t;
}

// Joint values of arm r at the lane's state (all loads first, so that they
// overlap).
__device__ __forceinline__ void arm_joints(const SceneDev &sc, const LaneState &st, int r, int nj,
                                           float (&qv)[kMaxJoints]) {
  const int q0 = as_const(sc.q_off)[r];
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

// One tile on the whole workgroup, then the edge flag (a colliding edge's
// flag word is set to hit_token; with skip_hit, states of an edge whose word
// already holds it are skipped); ends with a barrier (the tile's LDS is
// reused by the next one).
//
// With the joints' sines and cosines cached in LDS (sc_lds), the
// environment stage is balanced at run time: the waves first compute the
// joints' sines and cosines ((arm, joint) pairs spread over the waves, into
// LDS), then, after a barrier, claim (arm, link) jobs from an LDS counter in
// the order of decreasing link size, each composing its link's frame from the
// cached values and publishing the link's coarse centre.
// Without the cache, every wave runs whole chains for its (arm, link part)
// jobs.  Both end with a barrier before the arm-pair stage.
template <bool STAGED, bool CACHE>
__device__ void tile_work(const SceneDev &sc, const Src<STAGED> &src, int S, int w, int W, int lane, int it,
                          const TileLanes &tl, uint32_t *flags, float *cen, float *sc_lds, float *wave_fr,
                          uint32_t *wave_q, unsigned long long *s_dead, unsigned long long *s_hit, int *s_next,
                          WorkCount &wc, uint32_t &checked, uint32_t hit_token, bool skip_hit = false) {
  unsigned long long *const dead = &s_dead[it & 1];
  const LaneState &st = tl.st;
  bool act = tl.act;
  const int R = sc.n_robots;
  bool hit = false;
  // With skip_hit, a lane whose edge another tile of this launch has already
  // marked is idle, and hits are published at once (device-scope stores), so
  // that later tiles of the same edges can skip their states.  Waves may read
  // a word at different times; they then differ only on lanes of an edge
  // that is already marked, whose results no longer matter.
  if (skip_hit && act)
    act = __hip_atomic_load(&flags[tl.e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != hit_token;
  auto publish = [&]() {
    if (skip_hit && !hit) __hip_atomic_store(&flags[tl.e], hit_token, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    hit = true;
  };
  if constexpr (CACHE) {
    if (threadIdx.x == 0) *s_next = 0;
    // A. the joints' sines and cosines at every lane's state, (arm, joint)
    // pairs spread over the waves (a wave whose lanes are all idle has
    // nothing to compute: a lane is idle in every wave or on a marked edge)
    const int js_end = (!skip_hit || __ballot(act) != 0ull) ? R * kMaxJoints : 0;
    for (int js = w; js < js_end; js += W) {
      const int r = js / kMaxJoints, j = js - r * kMaxJoints;
      const int m = as_const(sc.model)[r];
      if (j >= as_const(sc.nj)[m]) continue;
      if (j == 0 && act) ++wc.chains;
      const float qj = joint_value(st, as_const(sc.q_off)[r] + j);
      float sn, cs;
      sincosf(qj + as_const(sc.theta_off)[m * kMaxJoints + j], &sn, &cs);
      float *q = sc_lds + ((r * kMaxJoints + j) * 2) * kWave + lane;
      q[0] = sn;
      q[kWave] = cs;
    }
    __syncthreads();
    const int n_jobs = R * kMaxLinks;
    for (;;) {
      int job = 0;
      if (lane == 0) job = atomicAdd(s_next, 1);
      job = __builtin_amdgcn_readfirstlane(__shfl(job, 0, kWave));
      if (job >= n_jobs) break;
      const int k = job / R, r = job - k * R;  // rank k of every arm, then rank k + 1
      const int m = as_const(sc.model)[r];
      const int l = as_const(sc.link_order)[m * kMaxLinks + k];
      if (l > as_const(sc.nj)[m]) continue;
      const bool live = act && !hit && !((dead_mask(dead) >> lane) & 1ull);
      if (__ballot(live) == 0ull) continue;
      // B. the link's frame from the cached values, its coarse centre
      // (published for the arm-pair stage), then its environment tests
      const Frame F = frame_cached(sc, r, m, l, lane, sc_lds);
      const float4 co = ld4(as_const(sc.coarse), m * kMaxLinks + l);
      const float3 c = apply(F, co.x, co.y, co.z);
      float *slot = cen + ((r * kMaxLinks + l) * 3) * kWave + lane;
      slot[0] = c.x;
      slot[kWave] = c.y;
      slot[2 * kWave] = c.z;
      if (link_env<STAGED>(sc, src, r, m, l, F, c, live, tl.emask, wave_fr, wave_q, &s_hit[w], dead, lane, wc))
        publish();
    }
  } else {
  for (int jb = w; jb < R * S; jb += W) {
    const int r = jb / S, part = jb - r * S;
    const int m = as_const(sc.model)[r];
    const int nj = as_const(sc.nj)[m];
    float qv[kMaxJoints];
    arm_joints(sc, st, r, nj, qv);
    const bool live = act && !hit;
    if (arm_env<STAGED>(sc, src, r, m, part, S, qv, live, tl.emask, cen, sc_lds, wave_fr, wave_q, &s_hit[w], dead,
                        lane, wc))
      publish();
  }
  }
  if (act && w == 0) ++checked;
  __syncthreads();
  if (threadIdx.x == 0) s_dead[(it + 1) & 1] = 0ull;  // last used by the previous tile
  // arm pairs that can reach each other
  if (arm_pairs<STAGED, CACHE>(sc, src, cen, sc_lds, w, W, act && !hit, st, tl.emask, wave_q, &s_hit[w], dead, lane, wc))
    hit = true;
  if (hit) {
    if (skip_hit) __hip_atomic_store(&flags[tl.e], hit_token, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else flags[tl.e] = hit_token;
  }
  __syncthreads();
}

// Workgroup totals of the work counters, one slot row per workgroup (summed
// by the final step; no device-wide atomics).  Each wave's sums go to its
// own row of `scratch` (LDS free by now, at least W kPartialSlots words), so
// no LDS atomics contend; one barrier, then one thread per slot adds the
// rows.
__device__ void write_partials(uint64_t *partials, uint32_t checked, uint32_t tiles, const WorkCount &wc, int w,
                               int W, int lane, unsigned long long *scratch) {
  const uint32_t v[kPartialSlots - 1] = {checked,      wc.chains, wc.links,  wc.env_tests, wc.box_exact,
                                         wc.rr_coarse, wc.fine_s, wc.fine_b, wc.fine_rr};
  uint64_t sum[kPartialSlots - 1];
#pragma unroll
  for (int i = 0; i < kPartialSlots - 1; ++i) sum[i] = wave_sum(v[i]);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < kPartialSlots - 1; ++i) scratch[w * kPartialSlots + i] = sum[i];
    scratch[w * kPartialSlots + kPartialSlots - 1] = w == 0 ? tiles : 0u;
  }
  __syncthreads();
  if (threadIdx.x < kPartialSlots) {
    unsigned long long t = 0;
    for (int u = 0; u < W; ++u) t += scratch[u * kPartialSlots + threadIdx.x];
    partials[(int64_t)blockIdx.x * kPartialSlots + threadIdx.x] = t;
  }
}

template <bool STAGED, bool CACHE>
__global__ __launch_bounds__(kWave * kMaxWavesPerBlock, 1) void validate_tiles_kernel(
    SceneDev sc, const float *__restrict__ qa, const float *__restrict__ qb, int64_t n_edges,
    const int64_t *__restrict__ off, const int32_t *__restrict__ tile_first, uint32_t *__restrict__ flags,
    uint64_t *__restrict__ counters, uint64_t *__restrict__ partials, int S) {
  // dynamic LDS: [R][kMaxLinks][3][64] published coarse centres, then per
  // wave kWaveLdsFloats (link frames, fine-test queue), then the staged scene
  extern __shared__ float cen[];
  // s_dead[t & 1]: lanes of tile t whose edge is known to collide (two
  // copies, so that the next tile's copy is cleared while this one is in use)
  __shared__ unsigned long long s_dead[2], s_hit[kMaxWavesPerBlock];
  __shared__ int s_next;  // next (arm, link) job of the tile
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
  if (threadIdx.x < 2) s_dead[threadIdx.x] = 0ull;
  float *const sc_lds = CACHE ? cen + (size_t)R * kMaxLinks * 3 * kWave : nullptr;
  float *const wave_fr = cen + tile_shared_floats(R, CACHE) + (size_t)w * kWaveLdsFloats;
  uint32_t *const wave_q = (uint32_t *)(wave_fr + 12 * kWave);
  const Src<STAGED> src = make_src<STAGED>(sc, cen + tile_shared_floats(R, CACHE) + (size_t)W * kWaveLdsFloats);
  // Workgroup b takes tiles b and b + G (G = grid) first; every further tile
  // comes from the launch's tile counter (counters[0], zeroed by the scan:
  // tiles 2G, 2G + 1, ...), so that workgroups whose tiles are light take
  // more of them.  The edge lookups run ahead: while a tile runs, the next
  // tile's lane offsets are loaded, and thread 0 claims the tile after it and
  // loads its first edge.  A tile is claimed only while the next one is
  // real, so every claimed tile below n_tiles is processed.
  __shared__ int64_t s_claim[2][2];  // (tile, first edge), two slots, alternating
  const int64_t G = gridDim.x;
  auto first_edge = [&](int64_t t) -> int64_t {
    return t < kTileFirstCap ? (int64_t)as_const(tile_first)[t] : find_edge(off, n_edges, t * kWave);
  };
  auto lane_off = [&](int64_t e_first) -> int64_t {
    const int64_t ei = e_first + lane < n_edges ? e_first + lane : n_edges;
    return off[ei];
  };
  int64_t tile = blockIdx.x, t_nxt = tile + G;
  int64_t e0_cur = first_edge(tile);
  int64_t off_cur = lane_off(e0_cur);
  int64_t e0_nxt = t_nxt < n_tiles ? first_edge(t_nxt) : 0;
  for (int it = 0; tile < n_tiles; ++it) {
    if (threadIdx.x == 0 && t_nxt < n_tiles) {
      const int64_t t = 2 * G + (int64_t)atomicAdd((unsigned long long *)&counters[0], 1ull);
      s_claim[it & 1][0] = t;
      s_claim[it & 1][1] = t < n_tiles ? first_edge(t) : 0;
    }
    const int64_t e0 = e0_cur, my_off = off_cur;
    if (t_nxt < n_tiles) {
      e0_cur = e0_nxt;
      off_cur = lane_off(e0_nxt);
    }
    if (w == 0) ++tiles;
    const TileLanes tl = map_lanes(tile * kWave, total, e0, my_off, off, 0, 0, qa, qb, sc.dof, lane);
    tile_work<STAGED, CACHE>(sc, src, S, w, W, lane, it, tl, flags, cen, sc_lds, wave_fr, wave_q, s_dead, s_hit, &s_next, wc,
                      checked, kFlagHit);
    // (the claim was written before tile_work's barriers)
    const int64_t t_nn = t_nxt < n_tiles ? s_claim[it & 1][0] : n_tiles;
    if (t_nxt < n_tiles) e0_nxt = s_claim[it & 1][1];
    tile = t_nxt;
    t_nxt = t_nn;
  }
  write_partials(partials, checked, tiles, wc, w, W, lane, (unsigned long long *)cen);
}

// ---------------------------------------------------------------------------
// 3b. small batches in one launch
// ---------------------------------------------------------------------------
//
// For at most kFusedMaxEdges edges whose state counts the producer of the
// edges has made (codes of state_count_code): every workgroup scans the
// counts into LDS itself, so no count and scan launches come first, and takes
// its tiles as the tile kernel does.  Colliding edges are marked with this
// launch's token, so flag words never need clearing between launches.  Only
// workgroups that hold a tile go on; the last of them to finish (a
// device-wide arrival counter) writes the bits and the counters and resets
// the counter: one launch where the general path makes three.  Workgroups
// never wait for each other.
// Word of the arrival buffer (256 bytes before the flag words, zero between
// launches) that hands out the small launches' tiles after the first.
constexpr int kTileCounterWord = 32;

template <bool STAGED, bool CACHE>
__global__ __launch_bounds__(kWave * kMaxWavesPerBlock, 1) void validate_small_kernel(
    SceneDev sc, const float *__restrict__ qa, const float *__restrict__ qb, int n_edges,
    const int32_t *__restrict__ codes, uint32_t *__restrict__ flags, uint32_t token, uint8_t *__restrict__ out,
    uint64_t *__restrict__ counters, uint64_t *__restrict__ partials, uint32_t *__restrict__ arrived,
    uint64_t *__restrict__ totals, int S) {
  extern __shared__ float cen[];
  __shared__ unsigned long long s_dead[2], s_hit[kMaxWavesPerBlock];
  __shared__ int s_next;  // next (arm, link) job of the tile
  __shared__ int64_t s_off[kFusedMaxEdges + 1];
  __shared__ unsigned long long s_sum[kPartialSlots + 3];
  __shared__ int s_last;
  __shared__ int64_t s_tile[2];  // the next tile, claimed during the current one (two slots, alternating)
  const int lane = threadIdx.x & (kWave - 1);
  const int w = (int)__builtin_amdgcn_readfirstlane(threadIdx.x / kWave), W = blockDim.x / kWave;
  const int R = sc.n_robots;
  // exclusive offsets of the counts in LDS (thread t sums edges [t k, t k + k))
  const int per = (n_edges + (int)blockDim.x - 1) / (int)blockDim.x;
  const int i0 = (int)threadIdx.x * per, i1 = min(i0 + per, n_edges);
  int64_t mine = 0;
  for (int i = i0; i < i1; ++i) mine += max(codes[i], 0);
  int64_t total_v;
  int64_t run = block_exclusive_scan(mine, &total_v);
  const int64_t total = (int64_t)uniform_u64((uint64_t)total_v);  // the same in every lane
  const int64_t n_tiles = (total + kWave - 1) / kWave;
  // More tiles than workgroups: two passes (map_lanes_split), the first, of
  // every K-th state, at most one tile per workgroup (it holds at most
  // total / K + n_edges states), so that the second pass's tiles mostly start
  // after the first pass has marked the colliding edges and skip their
  // states.  The segment offsets (2 n_edges + 1 words) take the place of the
  // plain offsets, so they need fewer than 2^31 states.
  const int64_t first_cap = (int64_t)gridDim.x * kWave - n_edges;
  const int K = (n_tiles > (int64_t)gridDim.x && first_cap > 0 && total <= (int64_t)INT32_MAX)
                    ? (int)max<int64_t>(2, (total + first_cap - 1) / first_cap)
                    : 1;
  int32_t *const s_seg = reinterpret_cast<int32_t *>(s_off);
  static_assert(sizeof(s_off) >= (2 * kFusedMaxEdges + 1) * sizeof(int32_t), "segment offsets fit");
  if (K > 1) {
    int64_t mine1 = 0;
    for (int i = i0; i < i1; ++i) mine1 += (max(codes[i], 0) + K - 1) / K;
    int64_t total1_v;
    int64_t run1 = block_exclusive_scan(mine1, &total1_v);
    const int64_t total1 = (int64_t)uniform_u64((uint64_t)total1_v);
    for (int i = i0; i < i1; ++i) {
      const int64_t c = max(codes[i], 0), c1 = (c + K - 1) / K;
      s_seg[i] = (int32_t)run1;
      s_seg[n_edges + i] = (int32_t)(total1 + run - run1);
      run += c;
      run1 += c1;
    }
    if (threadIdx.x == 0) s_seg[2 * n_edges] = (int32_t)total;
  } else {
    for (int i = i0; i < i1; ++i) {
      s_off[i] = run;
      run += max(codes[i], 0);
    }
    if (threadIdx.x == 0) s_off[n_edges] = total;
  }
  if (threadIdx.x < 2) s_dead[threadIdx.x] = 0ull;
  __syncthreads();
  // Workgroups with a tile take part (workgroup 0 when there is none); the
  // others leave now, so that a batch of few tiles pays for few arrivals and
  // partial sums.  Every workgroup computes the same count.
  const uint32_t working = (uint32_t)max<int64_t>(1, min<int64_t>((int64_t)gridDim.x, n_tiles));
  if (blockIdx.x >= working) return;
  if ((int64_t)blockIdx.x < n_tiles) {
    uint32_t checked = 0, tiles = 0;
    WorkCount wc;
    float *const sc_lds = CACHE ? cen + (size_t)R * kMaxLinks * 3 * kWave : nullptr;
    float *const wave_fr = cen + tile_shared_floats(R, CACHE) + (size_t)w * kWaveLdsFloats;
    uint32_t *const wave_q = (uint32_t *)(wave_fr + 12 * kWave);
    const Src<STAGED> src =
        make_src<STAGED>(sc, cen + tile_shared_floats(R, CACHE) + (size_t)W * kWaveLdsFloats);
    // Workgroup b first takes tile b; every further tile comes from the
    // launch's tile counter (tiles working, working + 1, ...), claimed by
    // thread 0 while the current tile runs, so that workgroups whose tiles
    // are light take more of them.  The last workgroup resets the counter.
    int it = 0;
    for (int64_t tile = blockIdx.x; tile < n_tiles; ++it) {
      if (threadIdx.x == 0) s_tile[it & 1] = (int64_t)working + atomicAdd(&arrived[kTileCounterWord], 1u);
      if (w == 0) ++tiles;
      TileLanes tl;
      if (K > 1) {
        const int64_t g0 = find_edge(s_seg, 2 * (int64_t)n_edges, tile * kWave);
        const int64_t my_off = s_seg[g0 + lane < 2 * n_edges ? g0 + lane : 2 * n_edges];
        tl = map_lanes_split(tile * kWave, total, g0, my_off, s_seg, n_edges, K, qa, qb, sc.dof, lane);
      } else {
        const int64_t e0 = find_edge(s_off, n_edges, tile * kWave);
        const int64_t my_off = s_off[e0 + lane < n_edges ? e0 + lane : n_edges];
        tl = map_lanes(tile * kWave, total, e0, my_off, s_off, 0, 0, qa, qb, sc.dof, lane);
      }
      tile_work<STAGED, CACHE>(sc, src, S, w, W, lane, it, tl, flags, cen, sc_lds, wave_fr, wave_q, s_dead, s_hit, &s_next, wc,
                        checked, token, K > 1);
      tile = s_tile[it & 1];  // written before tile_work's barriers
    }
    write_partials(partials, checked, tiles, wc, w, W, lane, (unsigned long long *)cen);
  } else if (threadIdx.x < kPartialSlots) {
    partials[(int64_t)blockIdx.x * kPartialSlots + threadIdx.x] = 0ull;
  }
  // Arrival.  Every wave waits until its own stores (flag words, partials)
  // are performed, the barrier orders them before thread 0's increment, and
  // that increment is an agent-scope release (an L2 write-back for the whole
  // workgroup's stores: one per workgroup instead of one per wave); the last
  // workgroup's waves acquire before reading what the others wrote.
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0)
    s_last = __hip_atomic_fetch_add(arrived, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == working - 1u;
  __syncthreads();
  if (!s_last) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  // The last workgroup: column sums of the partials and the bits with their
  // counts, every thread accumulating its share in registers; each wave's
  // sums go to its own row of LDS (free by now), then one thread per slot
  // adds the rows.
  constexpr int kCols = kPartialSlots + 3;  // then invalid, non-finite, too long
  uint64_t col[kCols] = {};
  for (int64_t k = threadIdx.x; k < (int64_t)working; k += blockDim.x) {
#pragma unroll
    for (int i = 0; i < kPartialSlots; ++i) col[i] += partials[k * kPartialSlots + i];
  }
  for (int e = threadIdx.x; e < n_edges; e += blockDim.x) {
    const int32_t c = codes[e];
    const bool ok = c > 0 && flags[e] != token;
    out[e] = ok ? 1 : 0;
    col[kPartialSlots] += ok ? 0 : 1;
    col[kPartialSlots + 1] += c == kCodeNonFinite ? 1 : 0;
    col[kPartialSlots + 2] += c == kCodeTooLong ? 1 : 0;
  }
  unsigned long long *const rows = (unsigned long long *)cen;
#pragma unroll
  for (int i = 0; i < kCols; ++i) {
    const uint64_t t = wave_sum(col[i]);
    if (lane == 0) rows[w * kCols + i] = t;
  }
  __syncthreads();
  if (threadIdx.x < kCols) {
    unsigned long long t = 0;
    for (int u = 0; u < W; ++u) t += rows[u * kCols + threadIdx.x];
    s_sum[threadIdx.x] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    counters[0] = 0;
    counters[1] = (uint64_t)total;
    counters[2] = s_sum[0];
    counters[3] = s_sum[kPartialSlots - 1];
    counters[4] = s_sum[kPartialSlots + 1];
    counters[5] = s_sum[kPartialSlots];
    counters[6] = s_sum[kPartialSlots + 2];
    counters[7] = 0;
    for (int i = 1; i < kPartialSlots - 1; ++i) counters[7 + i] = s_sum[i];
    if (totals) {
      totals[0] += s_sum[0];
      totals[1] += (uint64_t)total;
      for (int i = 1; i < kPartialSlots - 1; ++i) totals[1 + i] += s_sum[i];
    }
    *arrived = 0u;  // ready for the next launch
    arrived[kTileCounterWord] = 0u;
  }
}

// ---------------------------------------------------------------------------
// 4. many scenes in one launch (independent planning instances)
// ---------------------------------------------------------------------------
//
// The edges of all segments form one flat list; every segment's states are
// laid out from a tile boundary, so that a tile belongs to one segment (one
// scene, wave-uniform model data).  The tile table records each tile's
// segment and first edge.

// Segment of flat edge f (segments sorted by edge0).
__device__ __forceinline__ int seg_of_edge(const ValSeg *__restrict__ segs, int n_segs, int64_t f) {
  int lo = 0, hi = n_segs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].edge0 <= f) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(256) void seg_count_kernel(const ValSeg *__restrict__ segs, int n_segs, int64_t n_flat,
                                                        int32_t *__restrict__ n_out, uint32_t *__restrict__ flags,
                                                        int32_t *__restrict__ edge_seg) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n_flat) return;
  const int k = seg_of_edge(segs, n_segs, f);
  const ValSeg &g = segs[k];
  uint32_t fl;
  n_out[f] = edge_states(g.qa, g.qb, f - g.edge0, g.sc.dof, g.res, nullptr, &fl);
  flags[f] = fl;
  edge_seg[f] = k;
}

// Single workgroup: states and tiles of every segment, the first tile of
// each, the segments' counters (reset; [1] = edge states) and the total tile
// count (batch[1]; batch[2] = 1 when the tile table would overflow).
__global__ __launch_bounds__(kScanThreads) void seg_tiles_kernel(ValSeg *__restrict__ segs, int n_segs,
                                                                 const int64_t *__restrict__ off,
                                                                 uint64_t *__restrict__ batch) {
  int64_t carry = 0;
  for (int k0 = 0; k0 < n_segs; k0 += kScanThreads) {
    const int k = k0 + threadIdx.x;
    int64_t tiles = 0, states = 0;
    if (k < n_segs) {
      states = off[segs[k].edge0 + segs[k].n_edges] - off[segs[k].edge0];
      tiles = (states + kWave - 1) / kWave;
    }
    int64_t total;
    const int64_t ex = block_exclusive_scan(tiles, &total);
    if (k < n_segs) {
      segs[k].tile0 = carry + ex;
      uint64_t *c = segs[k].counters;
      for (int i = 0; i < 16; ++i) c[i] = 0;
      c[1] = (uint64_t)states;
    }
    carry += total;
  }
  if (threadIdx.x == 0) {
    batch[0] = 0;
    batch[1] = (uint64_t)carry;
    batch[2] = carry > kTileFirstCap ? 1 : 0;
    for (int c = 3; c < 16; ++c) batch[c] = 0;
  }
}

__global__ __launch_bounds__(256) void seg_table_kernel(const ValSeg *__restrict__ segs, int64_t n_flat,
                                                        const int32_t *__restrict__ n_states,
                                                        const int32_t *__restrict__ edge_seg,
                                                        const int64_t *__restrict__ off,
                                                        int32_t *__restrict__ tile_first, int32_t *__restrict__ tile_seg) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n_flat) return;
  const int k = edge_seg[f];
  const ValSeg &g = segs[k];
  const int64_t run = off[f] - off[g.edge0];
  const int64_t v = n_states[f];
  for (int64_t tl = (run + kWave - 1) / kWave; tl * kWave < run + v; ++tl) {
    const int64_t t = g.tile0 + tl;
    if (t >= kTileFirstCap) break;
    tile_first[t] = (int32_t)f;
    tile_seg[t] = k;
  }
}

template <bool CACHE>
__global__ __launch_bounds__(kWave * kMaxWavesPerBlock, 1) void validate_segments_kernel(
    const ValSeg *__restrict__ segs, const int64_t *__restrict__ off, const int32_t *__restrict__ tile_first,
    const int32_t *__restrict__ tile_seg, uint32_t *__restrict__ flags, uint64_t *__restrict__ batch,
    uint64_t *__restrict__ partials, int r_max) {
  extern __shared__ float cen[];
  __shared__ unsigned long long s_dead[2], s_hit[kMaxWavesPerBlock];
  __shared__ int s_next;  // next (arm, link) job of the tile
  const int lane = threadIdx.x & (kWave - 1);
  const int w = (int)__builtin_amdgcn_readfirstlane(threadIdx.x / kWave), W = blockDim.x / kWave;
  int64_t n_tiles = (int64_t)batch[1];
  if (batch[2]) n_tiles = 0;  // table overflow: reported by the host, nothing checked
  uint32_t checked = 0, tiles = 0;
  WorkCount wc;
  if ((int64_t)blockIdx.x >= n_tiles) {
    if (threadIdx.x < kPartialSlots) partials[(int64_t)blockIdx.x * kPartialSlots + threadIdx.x] = 0ull;
    return;
  }
  if (threadIdx.x < 2) s_dead[threadIdx.x] = 0ull;
  __syncthreads();
  float *const sc_lds = CACHE ? cen + (size_t)r_max * kMaxLinks * 3 * kWave : nullptr;
  float *const wave_fr = cen + tile_shared_floats(r_max, CACHE) + (size_t)w * kWaveLdsFloats;
  uint32_t *const wave_q = (uint32_t *)(wave_fr + 12 * kWave);
  // Workgroup b first takes tile b; every further tile comes from the
  // launch's tile counter (batch[0], zeroed by the table kernels: tiles G,
  // G + 1, ...), claimed by thread 0 while the current tile runs.
  __shared__ int64_t s_tile[2];  // the next tile, two slots, alternating
  const int64_t G = gridDim.x;
  int it = 0;
  for (int64_t tile = blockIdx.x; tile < n_tiles; ++it) {
    if (threadIdx.x == 0) s_tile[it & 1] = G + (int64_t)atomicAdd((unsigned long long *)&batch[0], 1ull);
    const int k = (int)__builtin_amdgcn_readfirstlane(tile_seg[tile]);
    const ValSeg &g = segs[k];
    const SceneDev &sc = g.sc;
    const Src<false> src = make_src<false>(sc, nullptr);
    const int64_t base = off[g.edge0], e_last = g.edge0 + g.n_edges;
    const int64_t e0 = tile_first[tile];
    const int64_t ei = e0 + lane < e_last ? e0 + lane : e_last;
    const int64_t my_off = off[ei] - base;
    const int64_t total = off[e_last] - base;
    if (w == 0) ++tiles;
    const TileLanes tl = map_lanes((tile - g.tile0) * kWave, total, e0, my_off, off, base, g.edge0, g.qa, g.qb,
                                   sc.dof, lane);
    tile_work<false, CACHE>(sc, src, g.S, w, W, lane, it, tl, flags, cen, sc_lds, wave_fr, wave_q, s_dead, s_hit, &s_next, wc,
                     checked, kFlagHit);
    tile = s_tile[it & 1];  // written before tile_work's barriers
  }
  write_partials(partials, checked, tiles, wc, w, W, lane, (unsigned long long *)cen);
}

// Bits of every segment's edges, their invalid counts, and (block 0) the
// work totals.
__global__ __launch_bounds__(256) void seg_finalize_kernel(const ValSeg *__restrict__ segs, int64_t n_flat,
                                                           const uint32_t *__restrict__ flags,
                                                           const int32_t *__restrict__ edge_seg,
                                                           const uint64_t *__restrict__ partials, int n_partials,
                                                           uint64_t *__restrict__ totals) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.x == 0 && totals) {
    __shared__ unsigned long long col[kPartialSlots];
    if (threadIdx.x < kPartialSlots) col[threadIdx.x] = 0ull;
    __syncthreads();
    uint64_t acc[kPartialSlots] = {};
    for (int b = threadIdx.x; b < n_partials; b += blockDim.x) {
#pragma unroll
      for (int i = 0; i < kPartialSlots; ++i) acc[i] += partials[(int64_t)b * kPartialSlots + i];
    }
#pragma unroll
    for (int i = 0; i < kPartialSlots; ++i) {
      for (int d = kWave / 2; d > 0; d >>= 1) acc[i] += __shfl_xor(acc[i], d, kWave);
      if ((threadIdx.x & (kWave - 1)) == 0) atomicAdd(&col[i], (unsigned long long)acc[i]);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      totals[0] += col[0];
      for (int i = 1; i < kPartialSlots - 1; ++i) totals[1 + i] += col[i];
    }
  }
  if (f >= n_flat) return;
  const int k = edge_seg[f];
  const ValSeg &g = segs[k];
  const uint32_t fl = flags[f];
  g.out[f - g.edge0] = fl == 0u ? 1 : 0;
  if (fl != 0u) atomicAdd((unsigned long long *)&g.counters[5], 1ull);
  if (f == g.edge0 && totals) atomicAdd((unsigned long long *)&totals[1], (unsigned long long)g.counters[1]);
}

// Zeroes one word (a tile counter, before a repeated tile launch).
__global__ void zero_word_kernel(uint64_t *p) { *p = 0ull; }

// Zeroes n flag words (before a repeated small launch with the same token).
__global__ __launch_bounds__(256) void zero_flags_kernel(uint32_t *p, int n) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i < n) p[i] = 0u;
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
    uint64_t acc[kPartialSlots] = {};
    for (int b = threadIdx.x; b < n_partials; b += blockDim.x) {
#pragma unroll
      for (int i = 0; i < kPartialSlots; ++i) acc[i] += partials[(int64_t)b * kPartialSlots + i];
    }
#pragma unroll
    for (int i = 0; i < kPartialSlots; ++i) {
      for (int d = kWave / 2; d > 0; d >>= 1) acc[i] += __shfl_xor(acc[i], d, kWave);
      if ((threadIdx.x & (kWave - 1)) == 0) atomicAdd(&col[i], (unsigned long long)acc[i]);
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

// Tile shape: S link parts per arm (waves per arm, up to one per link), W
// waves per workgroup,
// and whether the joint sines/cosines are cached in LDS for the arm-pair
// stage.  Small batches (few tiles, the planner's case) get the most waves
// per tile, so that a tile's latency shrinks; large batches keep two
// workgroups per CU.
struct TileShape {
  int S, W, cache_sc;
};

// Centres (and cached sines/cosines) of the tile plus every wave's frame and queue.
static size_t centre_lds_bytes(int n_robots, int W, int cache_sc) {
  return (tile_shared_floats(n_robots, cache_sc) + (size_t)W * kWaveLdsFloats) * sizeof(float);
}

// Dynamic LDS budget of the tile kernel: staging is used when the scene's
// copy fits next to the published centres.
constexpr size_t kLdsBudget = 150 * 1024;

// The rule for a workgroup of at most `cap` waves.
static TileShape tile_shape_cap(int n_robots, int cap) {
  int S = 1;
  while (S < kMaxLinks && n_robots * S * 2 <= cap) S *= 2;
  int W = std::min(n_robots * S, cap);
  while (W > 1 && centre_lds_bytes(n_robots, W, 0) > kLdsBudget) W /= 2;
  const int cache = centre_lds_bytes(n_robots, W, 1) <= kLdsBudget ? 1 : 0;
  return {S, W, cache};
}

static TileShape tile_shape(int n_robots, int64_t n_edges) {
  return tile_shape_cap(n_robots, n_edges <= kSmallBatchEdges ? kMaxWavesPerBlock : kMaxWavesPerBlock / 2);
}

// ---------------------------------------------------------------------------
// Tile-shape autotuner
// ---------------------------------------------------------------------------
//
// The waves per workgroup of the tile kernel are measured, not only ruled:
// the first launch of each kind -- (launch path, arms, spheres per arm,
// obstacles, batch-size bucket) -- runs the tile kernel once per candidate
// shape (at most 4, 8 and 16 waves), timed with events on the launch stream,
// and keeps the fastest.  Bits do not depend on the shape (each candidate
// makes the same decisions; the last run's stand).  Choices live in memory
// per process and, when a cache file is configured, in a JSON file of one
// entry per line that later processes load.
namespace {

struct TuneKey {
  int path, R, S, n_obs, bucket;
  bool operator<(const TuneKey &o) const {
    if (path != o.path) return path < o.path;
    if (R != o.R) return R < o.R;
    if (S != o.S) return S < o.S;
    if (n_obs != o.n_obs) return n_obs < o.n_obs;
    return bucket < o.bucket;
  }
};

struct Tuner {
  std::mutex mu;
  bool init = false, enabled = true;
  std::string file;
  std::map<TuneKey, int> table;  // key -> W

  void defaults_locked() {
    if (init) return;
    init = true;
    const char *e = std::getenv("MRPOP_AUTOTUNE");
    enabled = !(e && std::strcmp(e, "0") == 0);
    const char *f = std::getenv("MRPOP_TUNE_CACHE");
    file = f ? f : "";
    load_locked();
  }
  void load_locked() {
    if (file.empty()) return;
    FILE *fp = std::fopen(file.c_str(), "r");
    if (!fp) return;
    char line[512];
    while (std::fgets(line, sizeof line, fp)) {
      TuneKey k;
      int W = 0;
      char path[16] = {0};
      if (std::sscanf(line, " {\"path\": \"%15[a-z]\", \"arms\": %d, \"spheres\": %d, \"obstacles\": %d, "
                      "\"bucket\": %d, \"waves\": %d", path, &k.R, &k.S, &k.n_obs, &k.bucket, &W) == 6 &&
          W >= 1 && W <= kMaxWavesPerBlock) {
        k.path = std::strcmp(path, "small") == 0 ? 1 : std::strcmp(path, "general") == 0 ? 0 : -1;
        if (k.path >= 0) table[k] = W;
      }
    }
    std::fclose(fp);
  }
  void store_locked(const TuneKey &k, int W, const int *cand, const float *us, int n) {
    table[k] = W;
    if (file.empty()) return;
    FILE *fp = std::fopen(file.c_str(), "a");
    if (!fp) return;
    std::fprintf(fp, "{\"path\": \"%s\", \"arms\": %d, \"spheres\": %d, \"obstacles\": %d, \"bucket\": %d, "
                 "\"waves\": %d, \"measured_us\": {", k.path == 1 ? "small" : "general", k.R, k.S, k.n_obs,
                 k.bucket, W);
    for (int i = 0; i < n; ++i) std::fprintf(fp, "%s\"%d\": %.2f", i ? ", " : "", cand[i], us[i]);
    std::fprintf(fp, "}}\n");
    std::fclose(fp);
  }
};

Tuner &tuner() {
  static Tuner t;
  return t;
}

TuneKey tune_key(const SceneDev &sc, int64_t n_edges, int path) {
  int b = 0;
  while ((int64_t(1) << b) < n_edges && b < 62) ++b;
  return {path, sc.n_robots, sc.sph_stride, sc.n_env_spheres + sc.n_env_boxes, b};
}

}  // namespace

// Shape of a launch: the tuned one for its key, else the rule's (then, when
// tuning is on and `may_tune`, *cands gets the shapes to measure).
static TileShape chosen_shape(const SceneDev &sc, int64_t n_edges, int path, bool may_tune,
                              std::vector<TileShape> *cands, TuneKey *key) {
  const TileShape rule = tile_shape(sc.n_robots, n_edges);
  Tuner &T = tuner();
  std::lock_guard<std::mutex> lk(T.mu);
  T.defaults_locked();
  *key = tune_key(sc, n_edges, path);
  const auto it = T.table.find(*key);
  if (it != T.table.end()) {
    for (int cap : {4, 8, kMaxWavesPerBlock}) {
      const TileShape ts = tile_shape_cap(sc.n_robots, cap);
      if (ts.W == it->second) return ts;
    }
    return rule;
  }
  if (may_tune && T.enabled) {
    for (int cap : {4, 8, kMaxWavesPerBlock}) {
      const TileShape ts = tile_shape_cap(sc.n_robots, cap);
      bool seen = false;
      for (const TileShape &c : *cands) seen = seen || c.W == ts.W;
      if (!seen) cands->push_back(ts);
    }
    if (cands->size() < 2) cands->clear();
  }
  return rule;
}

static void tuned(const TuneKey &k, const std::vector<TileShape> &cands, const std::vector<float> &us) {
  int best = 0;
  for (size_t i = 1; i < us.size(); ++i)
    if (us[i] < us[best]) best = (int)i;
  std::vector<int> w;
  for (const TileShape &c : cands) w.push_back(c.W);
  Tuner &T = tuner();
  std::lock_guard<std::mutex> lk(T.mu);
  T.store_locked(k, cands[best].W, w.data(), us.data(), (int)us.size());
}

void tuner_configure(const char *cache_file, bool enable) {
  Tuner &T = tuner();
  std::lock_guard<std::mutex> lk(T.mu);
  T.init = true;
  T.enabled = enable;
  T.file = cache_file ? cache_file : "";
  T.table.clear();
  T.load_locked();
}

int tuner_entries() {
  Tuner &T = tuner();
  std::lock_guard<std::mutex> lk(T.mu);
  T.defaults_locked();
  return (int)T.table.size();
}

// LDS of one CU.
constexpr size_t kLdsPerCu = 160 * 1024;

// Staging in LDS: always under MRPOP_TILE_LDS when it fits; under
// MRPOP_TILE_AUTO only when it fits and does not lower the number of
// workgroups a CU holds (the scalar cache then serves the rows).
static bool use_staged(const SceneDev &sc, const TileShape &ts) {
  if (sc.tile_mode == MRPOP_TILE_SCALAR) return false;
  const size_t base = centre_lds_bytes(sc.n_robots, ts.W, ts.cache_sc);
  const size_t staged = base + staged_floats(sc) * sizeof(float);
  if (staged > kLdsBudget) return false;
  if (sc.tile_mode == MRPOP_TILE_LDS) return true;
  return kLdsPerCu / staged >= kLdsPerCu / base;
}

// Calls go(staged, cache) with both as compile-time constants
// (std::integral_constant), one kernel instance per combination.
template <class Go>
static void dispatch_tile(bool staged, bool cache, Go &&go) {
  using T = std::true_type;
  using F = std::false_type;
  if (staged) {
    if (cache) go(T{}, T{});
    else go(T{}, F{});
  } else {
    if (cache) go(F{}, T{});
    else go(F{}, F{});
  }
}

// Resident workgroups for a persistent launch (cached per block size, staging
// and LDS size).
template <bool STAGED, bool CACHE>
static int persistent_grid(int W, size_t lds) {
  struct Key {
    int w;
    size_t lds;
    int grid;
  };
  static std::vector<Key> cache;
  for (const Key &k : cache)
    if (k.w == W && k.lds == lds) return k.grid;
  int dev = 0, cus = 0, per = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, validate_tiles_kernel<STAGED, CACHE>, kWave * W, lds);
  const int grid = std::min(kMaxGrid, std::max(1, cus) * std::max(1, per));
  cache.push_back({W, lds, grid});
  return grid;
}

static bool capturing(hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone;
}

// Runs launch(shape, start, stop) for every candidate, timing each with its
// own events (the caller's event pair, if any, on the last one), and records
// the fastest for `key`.  Waits for the stream.
template <class Launch>
static hipError_t time_candidates(const std::vector<TileShape> &cands, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                                  Launch &&launch, const TuneKey &key) {
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  std::vector<float> us;
  for (size_t i = 0; i < cands.size() && e == hipSuccess; ++i) {
    const bool last = i + 1 == cands.size();
    e = hipEventRecord(a, s);
    if (e != hipSuccess) break;
    launch(cands[i], last ? e0 : nullptr, last ? e1 : nullptr);
    if ((e = hipGetLastError()) != hipSuccess) break;
    if ((e = hipEventRecord(b, s)) != hipSuccess) break;
    if ((e = hipEventSynchronize(b)) != hipSuccess) break;
    float ms = 0.f;
    if ((e = hipEventElapsedTime(&ms, a, b)) != hipSuccess) break;
    us.push_back(ms * 1e3f);
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (e == hipSuccess) tuned(key, cands, us);
  return e;
}

hipError_t launch_validate(const SceneDev &sc, const float *qa, const float *qb, int64_t n_edges, float res,
                           const int32_t *n_states_opt, uint8_t *out_valid, const ValidateScratch &ws,
                           hipStream_t s, const std::pair<hipEvent_t, hipEvent_t> *ev_pair, uint64_t *totals,
                           int32_t *grid_out, int32_t *block_out, bool may_tune) {
  const int64_t nb = scan_blocks(n_edges);
  const int64_t g256 = (n_edges + 255) / 256;
  if (g256 > 0x7fffffff || nb > 0x7fffffff) return hipErrorInvalidValue;
  if (small_scan(n_edges, sc.dof)) {
    hipLaunchKernelGGL(count_scan_small_kernel, dim3(1), dim3(kScanThreads), 0, s, qa, qb, n_edges, sc.dof, res,
                       n_states_opt, ws.n_states, ws.flags, ws.offsets, ws.tile_first, ws.counters);
  } else {
    hipLaunchKernelGGL(count_states_kernel, dim3((unsigned)g256), dim3(256), 0, s, qa, qb, n_edges, sc.dof, res,
                       n_states_opt, ws.n_states, ws.flags);
    hipLaunchKernelGGL(scan_partials_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, s, ws.n_states, n_edges,
                       ws.block_sums);
    hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(kScanThreads), 0, s, ws.block_sums, nb, ws.counters);
    hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, s, ws.n_states, n_edges,
                       ws.block_sums, ws.offsets, ws.tile_first);
  }
  std::vector<TileShape> cands;
  TuneKey key;
  const TileShape ts0 = chosen_shape(sc, n_edges, 0, may_tune && !capturing(s), &cands, &key);
  // with events: recorded by the dispatch itself, at the kernel's start and end
  hipEvent_t e0 = ev_pair ? ev_pair->first : nullptr, e1 = ev_pair ? ev_pair->second : nullptr;
  int grid = 0;
  auto launch_tiles = [&](const TileShape &ts, hipEvent_t a, hipEvent_t b) {
    const bool staged = use_staged(sc, ts);
    const size_t lds =
        centre_lds_bytes(sc.n_robots, ts.W, ts.cache_sc) + (staged ? staged_floats(sc) * sizeof(float) : 0);
    auto go = [&](auto staged_c, auto cache_c) {
      constexpr bool ST = decltype(staged_c)::value, CA = decltype(cache_c)::value;
      grid = persistent_grid<ST, CA>(ts.W, lds);
      hipExtLaunchKernelGGL(validate_tiles_kernel<ST, CA>, dim3(grid), dim3(kWave * ts.W), (uint32_t)lds, s, a, b,
                            0, sc, qa, qb, n_edges, ws.offsets, ws.tile_first, ws.flags, ws.counters, ws.partials,
                            ts.S);
    };
    dispatch_tile(staged, ts.cache_sc != 0, go);
    if (block_out) *block_out = kWave * ts.W;
  };
  if (cands.empty()) {
    launch_tiles(ts0, e0, e1);
  } else {  // measured: every candidate once (the flag words only gather hits), the last one's partials stand
    const hipError_t te = time_candidates(cands, s, e0, e1, [&](const TileShape &ts, hipEvent_t a, hipEvent_t b) {
      // each candidate hands out every tile again: its tile counter starts at zero
      hipLaunchKernelGGL(zero_word_kernel, dim3(1), dim3(1), 0, s, ws.counters);
      launch_tiles(ts, a, b);
    }, key);
    if (te != hipSuccess) return te;
  }
  if (grid_out) *grid_out = grid;
  hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)g256), dim3(256), 0, s, ws.flags, n_edges, out_valid,
                     ws.counters, ws.partials, grid, totals);
  return hipGetLastError();
}

template <bool STAGED, bool CACHE>
static int small_grid(int W, size_t lds) {
  struct Key {
    int w;
    size_t lds;
    int grid;
  };
  static std::vector<Key> cache;
  for (const Key &k : cache)
    if (k.w == W && k.lds == lds) return k.grid;
  int dev = 0, cus = 0, per = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, validate_small_kernel<STAGED, CACHE>, kWave * W, lds);
  // At most two workgroups per CU: every workgroup scans the counts and
  // arrives once, and the last one reads every workgroup's partial sums, so
  // idle workgroups (small waves of one-arm scenes fit many per CU) cost time.
  const int grid = std::min(kMaxGrid, std::max(1, cus) * std::min(2, std::max(1, per)));
  cache.push_back({W, lds, grid});
  return grid;
}

hipError_t launch_validate_small(const SceneDev &sc, const float *qa, const float *qb, int64_t n_edges,
                                 const int32_t *codes, uint8_t *out_valid, const ValidateScratch &ws,
                                 uint32_t *arrived, uint32_t token, hipStream_t s,
                                 const std::pair<hipEvent_t, hipEvent_t> *ev_pair, uint64_t *totals,
                                 int32_t *grid_out, int32_t *block_out) {
  if (n_edges <= 0 || n_edges > kFusedMaxEdges || !codes || !arrived || (token & 0x80000000u) == 0u)
    return hipErrorInvalidValue;
  std::vector<TileShape> cands;
  TuneKey key;
  const TileShape ts0 = chosen_shape(sc, n_edges, 1, !capturing(s), &cands, &key);
  hipEvent_t e0 = ev_pair ? ev_pair->first : nullptr, e1 = ev_pair ? ev_pair->second : nullptr;
  int grid = 0;
  auto launch_small = [&](const TileShape &ts, hipEvent_t a, hipEvent_t b) {
    const bool staged = use_staged(sc, ts);
    const size_t lds =
        centre_lds_bytes(sc.n_robots, ts.W, ts.cache_sc) + (staged ? staged_floats(sc) * sizeof(float) : 0);
    auto go = [&](auto staged_c, auto cache_c) {
      constexpr bool ST = decltype(staged_c)::value, CA = decltype(cache_c)::value;
      grid = small_grid<ST, CA>(ts.W, lds);
      hipExtLaunchKernelGGL(validate_small_kernel<ST, CA>, dim3(grid), dim3(kWave * ts.W), (uint32_t)lds, s, a, b,
                            0, sc, qa, qb, (int)n_edges, codes, ws.flags, token, out_valid, ws.counters,
                            ws.partials, arrived, totals, ts.S);
    };
    dispatch_tile(staged, ts.cache_sc != 0, go);
    if (block_out) *block_out = kWave * ts.W;
  };
  if (cands.empty()) {
    launch_small(ts0, e0, e1);
  } else {  // measured: each candidate is a whole validation; the last one's bits and counters stand
    // Every candidate starts from cleared flag words: the two-pass order
    // skips the states of edges whose word holds the token, which an
    // earlier candidate would have set.
    const unsigned zb = (unsigned)((n_edges + 255) / 256);
    const hipError_t te = time_candidates(cands, s, e0, e1, [&](const TileShape &ts, hipEvent_t a, hipEvent_t b) {
      hipLaunchKernelGGL(zero_flags_kernel, dim3(zb), dim3(256), 0, s, ws.flags, (int)n_edges);
      launch_small(ts, a, b);
    }, key);
    if (te != hipSuccess) return te;
  }
  if (grid_out) *grid_out = grid;
  return hipGetLastError();
}

size_t seg_scratch_bytes(int64_t n_flat) {
  size_t b = 0;
  auto add = [&](size_t n) {
    b = (b + 255) & ~size_t(255);
    b += n;
  };
  add(sizeof(int32_t) * n_flat);
  add(sizeof(int32_t) * n_flat);
  add(sizeof(uint32_t) * n_flat);
  add(sizeof(int64_t) * (n_flat + 1));
  add(sizeof(int64_t) * (scan_blocks(n_flat) + 1));
  add(sizeof(uint64_t) * 16);
  add(sizeof(uint64_t) * kPartialSlots * kMaxGrid);
  add(sizeof(int32_t) * kTileFirstCap);
  add(sizeof(int32_t) * kTileFirstCap);
  return b + 256;
}

SegScratch seg_scratch_layout(void *base, int64_t n_flat) {
  size_t b = 0;
  auto take = [&](size_t n) {
    b = (b + 255) & ~size_t(255);
    void *p = (unsigned char *)base + b;
    b += n;
    return p;
  };
  SegScratch w;
  w.n_states = (int32_t *)take(sizeof(int32_t) * n_flat);
  w.edge_seg = (int32_t *)take(sizeof(int32_t) * n_flat);
  w.flags = (uint32_t *)take(sizeof(uint32_t) * n_flat);
  w.offsets = (int64_t *)take(sizeof(int64_t) * (n_flat + 1));
  w.block_sums = (int64_t *)take(sizeof(int64_t) * (scan_blocks(n_flat) + 1));
  w.batch = (uint64_t *)take(sizeof(uint64_t) * 16);
  w.partials = (uint64_t *)take(sizeof(uint64_t) * kPartialSlots * kMaxGrid);
  w.tile_first = (int32_t *)take(sizeof(int32_t) * kTileFirstCap);
  w.tile_seg = (int32_t *)take(sizeof(int32_t) * kTileFirstCap);
  return w;
}

int seg_link_split(int n_robots, int W) {
  int S = 1;
  while (S < kMaxLinks && n_robots * S * 2 <= W) S *= 2;
  return S;
}

void seg_shape(int r_max, int64_t n_flat, int *W, int *cache_sc) {
  const TileShape ts = tile_shape(r_max, n_flat);
  *W = ts.W;
  *cache_sc = ts.cache_sc;
}

template <bool CACHE>
static int segments_grid(int W, size_t lds) {
  struct Key {
    int w;
    size_t lds;
    int grid;
  };
  static std::vector<Key> cache;
  for (const Key &k : cache)
    if (k.w == W && k.lds == lds) return k.grid;
  int dev = 0, cus = 0, per = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, validate_segments_kernel<CACHE>, kWave * W, lds);
  const int grid = std::min(kMaxGrid, std::max(1, cus) * std::max(1, per));
  cache.push_back({W, lds, grid});
  return grid;
}

// The tile and final kernels of a many-scene launch (tables already built).
static hipError_t launch_segments_tail(const ValSeg *d_segs, int r_max, int64_t n_flat, const SegScratch &ws,
                                       hipStream_t s, const std::pair<hipEvent_t, hipEvent_t> *ev_pair,
                                       uint64_t *totals, int32_t *grid_out, int32_t *block_out) {
  const int64_t g256 = (n_flat + 255) / 256;
  int W = 0, cache = 0;
  seg_shape(r_max, n_flat, &W, &cache);
  const size_t lds = centre_lds_bytes(r_max, W, cache);
  hipEvent_t e0 = ev_pair ? ev_pair->first : nullptr, e1 = ev_pair ? ev_pair->second : nullptr;
  int grid = 0;
  auto go = [&](auto, auto cache_c) {
    constexpr bool CA = decltype(cache_c)::value;
    grid = segments_grid<CA>(W, lds);
    hipExtLaunchKernelGGL(validate_segments_kernel<CA>, dim3(grid), dim3(kWave * W), (uint32_t)lds, s, e0, e1, 0,
                          d_segs, ws.offsets, ws.tile_first, ws.tile_seg, ws.flags, ws.batch, ws.partials, r_max);
  };
  dispatch_tile(false, cache != 0, go);
  if (grid_out) *grid_out = grid;
  if (block_out) *block_out = kWave * W;
  hipLaunchKernelGGL(seg_finalize_kernel, dim3((unsigned)g256), dim3(256), 0, s, d_segs, n_flat, ws.flags,
                     ws.edge_seg, ws.partials, grid, totals);
  return hipGetLastError();
}

hipError_t launch_validate_segments(ValSeg *d_segs, int n_segs, int r_max, int64_t n_flat, const SegScratch &ws,
                                    hipStream_t s, const std::pair<hipEvent_t, hipEvent_t> *ev_pair,
                                    uint64_t *totals, int32_t *grid_out, int32_t *block_out) {
  if (n_segs <= 0 || n_flat <= 0) return hipSuccess;
  const int64_t nb = scan_blocks(n_flat);
  const int64_t g256 = (n_flat + 255) / 256;
  if (g256 > 0x7fffffff || nb > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(seg_count_kernel, dim3((unsigned)g256), dim3(256), 0, s, d_segs, n_segs, n_flat, ws.n_states,
                     ws.flags, ws.edge_seg);
  hipLaunchKernelGGL(scan_partials_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, s, ws.n_states, n_flat,
                     ws.block_sums);
  hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(kScanThreads), 0, s, ws.block_sums, nb, ws.batch);
  hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, s, ws.n_states, n_flat,
                     ws.block_sums, ws.offsets, (int32_t *)nullptr);
  hipLaunchKernelGGL(seg_tiles_kernel, dim3(1), dim3(kScanThreads), 0, s, d_segs, n_segs, ws.offsets, ws.batch);
  hipLaunchKernelGGL(seg_table_kernel, dim3((unsigned)g256), dim3(256), 0, s, d_segs, n_flat, ws.n_states,
                     ws.edge_seg, ws.offsets, ws.tile_first, ws.tile_seg);
  return launch_segments_tail(d_segs, r_max, n_flat, ws, s, ev_pair, totals, grid_out, block_out);
}

hipError_t launch_validate_segments_small(const ValSeg *segs, int n_segs, int r_max, int64_t n_flat, ValSeg *d_segs,
                                          const SegScratch &ws, hipStream_t s,
                                          const std::pair<hipEvent_t, hipEvent_t> *ev_pair, uint64_t *totals,
                                          int32_t *grid_out, int32_t *block_out) {
  if (n_segs <= 0 || n_flat <= 0) return hipSuccess;
  if (n_segs > kSegSmallMax || n_flat > kSmallScanEdges) return hipErrorInvalidValue;
  int64_t e = 0;
  for (int k = 0; k < n_segs; ++k) {  // consecutive, in order, covering [0, n_flat)
    if (segs[k].edge0 != e || segs[k].n_edges < 0) return hipErrorInvalidValue;
    e += segs[k].n_edges;
  }
  if (e != n_flat) return hipErrorInvalidValue;
  SegSmall in;
  std::memset(&in, 0, sizeof(in));
  for (int k = 0; k < n_segs; ++k) in.s[k] = segs[k];
  hipLaunchKernelGGL(seg_prep_small_kernel, dim3(1), dim3(kScanThreads), 0, s, in, n_segs, n_flat, d_segs,
                     ws.n_states, ws.flags, ws.edge_seg, ws.offsets, ws.tile_first, ws.tile_seg, ws.batch);
  return launch_segments_tail(d_segs, r_max, n_flat, ws, s, ev_pair, totals, grid_out, block_out);
}

}  // namespace mrpop
