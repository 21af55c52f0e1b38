// Composite edge validation: state counts, prefix scan, and the tile kernel.
//
// An edge (q_a, q_b) is checked at n discretised states (paper, Sec.
// "Multi-Thread Reassignment for Collision Checking").  The states of all
// edges form one global list (exclusive prefix sum of the per-edge counts);
// persistent waves pull fixed-size tiles of that list from an atomic queue.
//
// Lane mapping inside a wave (64 lanes): lane = (state t, arm r), so a wave
// holds T = floor(64 / R) states of up to 64/R consecutive list positions and
// every lane runs exactly one kinematic chain.  Per lane, link by link:
//   1. compose the link frame (modified DH), keep it in registers and, when
//      several arms share the state, publish it in LDS;
//   2. coarse test: the link's bounding sphere against every environment
//      sphere and box (wave-uniform obstacle loop, scalar loads);
//   3. fine test: only for flagged (link, obstacle) pairs, the link's spheres
//      against that obstacle.
// Then arm-arm pairs of the same state are split round-robin over the lanes
// of that state: coarse link-link tests on sphere centres rebuilt from the
// partner's frames in LDS, and fine sphere-sphere tests for flagged pairs.
// A collision marks the edge in a flag word; lanes whose edge is already
// marked skip their state (early exit across tiles), and lanes of a state
// that another lane found colliding skip the arm-arm phase.
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
  add(sizeof(uint64_t) * 8);
  add(sizeof(int64_t) * (scan_blocks(n_edges) + 1));
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
  w.counters = (uint64_t *)take(sizeof(uint64_t) * 8);
  w.block_sums = (int64_t *)take(sizeof(int64_t) * (scan_blocks(n_edges) + 1));
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
    for (int c = 2; c < 8; ++c) counters[c] = 0;
  }
}

__global__ __launch_bounds__(kScanThreads) void scan_apply_kernel(const int32_t *__restrict__ n, int64_t n_edges,
                                                                  const int64_t *__restrict__ block_sums,
                                                                  int64_t *__restrict__ offsets) {
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
    if (base + i < n_edges) offsets[base + i] = run;
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

// Coarse-then-fine environment test of one link whose frame is F.
__device__ __forceinline__ bool env_link(const SceneDev &sc, int m, int l, const Frame &F) {
  const float4 cs = sc.coarse[m * kMaxLinks + l];
  if (cs.w < 0.f) return false;
  const float3 c = apply(F, cs.x, cs.y, cs.z);
  const int32_t *ls = sc.link_start + m * (kMaxLinks + 1);
  const int i0 = ls[l], i1 = ls[l + 1];
  const float4 *fine = sc.fine + (int64_t)m * sc.sph_stride;
  for (int k = 0; k < sc.n_env_spheres; ++k) {
    const float4 o = sc.env_s[k];
    const float rs = cs.w + o.w;
    if (dist2(c, o) < rs * rs) {
      for (int i = i0; i < i1; ++i) {
        const float4 p = fine[i];
        const float3 w = apply(F, p.x, p.y, p.z);
        const float rr = p.w + o.w;
        if (dist2(w, o) < rr * rr) return true;
      }
    }
  }
  const float cr2 = cs.w * cs.w;
  for (int k = 0; k < sc.n_env_boxes; ++k) {
    const float4 lo = sc.env_b[2 * k], hi = sc.env_b[2 * k + 1];
    if (box_dist2(c, lo, hi) < cr2) {
      for (int i = i0; i < i1; ++i) {
        const float4 p = fine[i];
        const float3 w = apply(F, p.x, p.y, p.z);
        if (box_dist2(w, lo, hi) < p.w * p.w) return true;
      }
    }
  }
  return false;
}

// Frame of link l of the arm run by lane `ln`: the base for l == 0, else the
// copy the lane published in LDS (layout [link-1][component][lane]).
__device__ __forceinline__ Frame frame_of(const SceneDev &sc, const float *lds, int robot, int ln, int l) {
  if (l == 0) return load_frame(sc.base + 12 * robot);
  const float *p = lds + (l - 1) * 12 * kWave + ln;
  Frame f;
  f.r00 = p[0 * kWave]; f.r01 = p[1 * kWave]; f.r02 = p[2 * kWave]; f.t0 = p[3 * kWave];
  f.r10 = p[4 * kWave]; f.r11 = p[5 * kWave]; f.r12 = p[6 * kWave]; f.t1 = p[7 * kWave];
  f.r20 = p[8 * kWave]; f.r21 = p[9 * kWave]; f.r22 = p[10 * kWave]; f.t2 = p[11 * kWave];
  return f;
}

// Arm-arm test between this lane's arm (robot r, model m, lane ln) and the
// partner (robot p, model mp, lane pl) at the same state.
__device__ bool pair_test(const SceneDev &sc, const float *lds, int r, int m, int ln, int p, int mp, int pl) {
  const int nja = sc.nj[m], njb = sc.nj[mp];
  float3 cb[kMaxLinks];
  float rb[kMaxLinks];
#pragma unroll
  for (int b = 0; b < kMaxLinks; ++b) {
    rb[b] = -1.f;
    cb[b] = make_float3(0.f, 0.f, 0.f);
    if (b <= njb) {
      const float4 cs = sc.coarse[mp * kMaxLinks + b];
      const Frame F = frame_of(sc, lds, p, pl, b);
      cb[b] = apply(F, cs.x, cs.y, cs.z);
      rb[b] = cs.w;
    }
  }
  uint64_t flagged = 0;
#pragma unroll
  for (int a = 0; a < kMaxLinks; ++a) {
    if (a > nja) continue;
    const float4 cs = sc.coarse[m * kMaxLinks + a];
    if (cs.w < 0.f) continue;
    const Frame F = frame_of(sc, lds, r, ln, a);
    const float3 ca = apply(F, cs.x, cs.y, cs.z);
#pragma unroll
    for (int b = 0; b < kMaxLinks; ++b) {
      const float rs = cs.w + rb[b];
      if (rb[b] >= 0.f && dist2(ca, cb[b]) < rs * rs) flagged |= 1ull << (a * kMaxLinks + b);
    }
  }
  const int32_t *lsa = sc.link_start + m * (kMaxLinks + 1), *lsb = sc.link_start + mp * (kMaxLinks + 1);
  const float4 *fa = sc.fine + (int64_t)m * sc.sph_stride, *fb = sc.fine + (int64_t)mp * sc.sph_stride;
  while (flagged) {
    const int bit = __ffsll((unsigned long long)flagged) - 1;
    flagged &= flagged - 1;
    const int a = bit / kMaxLinks, b = bit - a * kMaxLinks;
    const Frame Fa = frame_of(sc, lds, r, ln, a), Fb = frame_of(sc, lds, p, pl, b);
    for (int i = lsa[a]; i < lsa[a + 1]; ++i) {
      const float4 pa = fa[i];
      const float3 wa = apply(Fa, pa.x, pa.y, pa.z);
      for (int j = lsb[b]; j < lsb[b + 1]; ++j) {
        const float4 pb = fb[j];
        const float3 wb = apply(Fb, pb.x, pb.y, pb.z);
        const float rs = pa.w + pb.w;
        if (dist2(wa, wb) < rs * rs) return true;
      }
    }
  }
  return false;
}

template <bool HOMOG, bool MULTI>
__global__ __launch_bounds__(kWave) void validate_tiles_kernel(SceneDev sc, const float *__restrict__ qa,
                                                               const float *__restrict__ qb, int64_t n_edges,
                                                               const int32_t *__restrict__ nst,
                                                               const int64_t *__restrict__ off,
                                                               uint32_t *__restrict__ flags,
                                                               uint64_t *__restrict__ counters) {
  __shared__ float lds[MULTI ? kMaxJoints * 12 * kWave : 1];
  const int lane = threadIdx.x;
  const int R = sc.n_robots;
  const int T = MULTI ? kWave / R : kWave;
  const int t = MULTI ? lane / R : lane;
  const int r = MULTI ? lane - t * R : 0;
  const bool slot_ok = t < T;
  const int m = HOMOG ? 0 : sc.model[r];
  const int nj = sc.nj[m];
  const int64_t total = (int64_t)counters[1];
  uint32_t checked = 0, tiles = 0;
  for (;;) {
    uint64_t tile = 0;
    if (lane == 0) tile = atomicAdd((unsigned long long *)&counters[0], 1ull);
    tile = uniform_u64(tile);
    const int64_t s0 = (int64_t)tile * T;
    if (s0 >= total) break;
    ++tiles;
    const int64_t s = s0 + t;
    bool act = slot_ok && s < total;
    int64_t e = 0;
    float tt = 0.f;
    bool last = false;
    if (act) {
      e = find_edge(off, n_edges, s);
      const int k = (int)(s - off[e]);
      const int n = nst[e];
      last = n > 1 && k == n - 1;
      tt = n > 1 ? (float)k / (float)(n - 1) : 0.f;
      if (load_relaxed(flags + e) != 0u) act = false;
    }
    if (act && r == 0) ++checked;
    const float *pa = qa + e * sc.dof + sc.q_off[r];
    const float *pb = qb + e * sc.dof + sc.q_off[r];
    Frame F = load_frame(sc.base + 12 * r);
    bool hit = act && env_link(sc, m, 0, F);
    for (int j = 1; j <= nj; ++j) {
      const float a = pa[j - 1], b = pb[j - 1];
      const float qj = last ? b : fmaf(tt, b - a, a);
      joint_step(F, sc.dh[m * kMaxJoints + j - 1], qj + sc.theta_off[m * kMaxJoints + j - 1]);
      if (MULTI) {
        float *o = lds + (j - 1) * 12 * kWave + lane;
        o[0 * kWave] = F.r00; o[1 * kWave] = F.r01; o[2 * kWave] = F.r02; o[3 * kWave] = F.t0;
        o[4 * kWave] = F.r10; o[5 * kWave] = F.r11; o[6 * kWave] = F.r12; o[7 * kWave] = F.t1;
        o[8 * kWave] = F.r20; o[9 * kWave] = F.r21; o[10 * kWave] = F.r22; o[11 * kWave] = F.t2;
      }
      if (act && !hit) hit = env_link(sc, m, j, F);
    }
    if (MULTI) {
      __syncthreads();
      const uint64_t hm = __ballot(hit);
      const uint64_t group = (R >= 64 ? ~0ull : ((1ull << R) - 1ull)) << (t * R);
      const bool state_dead = slot_ok && (hm & group) != 0ull;
      if (act && !state_dead) {
        const int npart = (R - 1) / 2 + ((R % 2 == 0 && r < R / 2) ? 1 : 0);
        for (int kk = 1; kk <= npart && !hit; ++kk) {
          int p = r + kk;
          if (p >= R) p -= R;
          const int mp = HOMOG ? 0 : sc.model[p];
          hit = pair_test(sc, lds, r, m, lane, p, mp, t * R + p);
        }
      }
      __syncthreads();
    }
    if (hit) flags[e] = kFlagHit;
  }
  // wave totals of the work counters
  for (int d = kWave / 2; d > 0; d >>= 1) checked += __shfl_xor(checked, d, kWave);
  if (lane == 0) {
    atomicAdd((unsigned long long *)&counters[2], (unsigned long long)checked);
    atomicAdd((unsigned long long *)&counters[3], (unsigned long long)tiles);
  }
}

__global__ __launch_bounds__(256) void finalize_kernel(const uint32_t *__restrict__ flags, int64_t n_edges,
                                                       uint8_t *__restrict__ out, uint64_t *__restrict__ counters) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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

template <bool HOMOG, bool MULTI>
static int persistent_grid() {
  static int grid = 0;
  if (grid == 0) {
    int dev = 0, cus = 0, per = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, validate_tiles_kernel<HOMOG, MULTI>, kWave, 0);
    grid = std::max(1, cus) * std::max(1, per);
  }
  return grid;
}

hipError_t launch_validate(const SceneDev &sc, const float *qa, const float *qb, int64_t n_edges, float res,
                           const int32_t *n_states_opt, uint8_t *out_valid, const ValidateScratch &ws,
                           hipStream_t s) {
  const int64_t nb = scan_blocks(n_edges);
  const int64_t g256 = (n_edges + 255) / 256;
  if (g256 > 0x7fffffff || nb > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(count_states_kernel, dim3((unsigned)g256), dim3(256), 0, s, qa, qb, n_edges, sc.dof, res,
                     n_states_opt, ws.n_states, ws.flags);
  hipLaunchKernelGGL(scan_partials_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, s, ws.n_states, n_edges,
                     ws.block_sums);
  hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(kScanThreads), 0, s, ws.block_sums, nb, ws.counters);
  hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, s, ws.n_states, n_edges,
                     ws.block_sums, ws.offsets);
  const bool multi = sc.n_robots > 1;
  if (sc.homogeneous) {
    if (multi)
      hipLaunchKernelGGL((validate_tiles_kernel<true, true>), dim3(persistent_grid<true, true>()), dim3(kWave), 0, s,
                         sc, qa, qb, n_edges, ws.n_states, ws.offsets, ws.flags, ws.counters);
    else
      hipLaunchKernelGGL((validate_tiles_kernel<true, false>), dim3(persistent_grid<true, false>()), dim3(kWave), 0,
                         s, sc, qa, qb, n_edges, ws.n_states, ws.offsets, ws.flags, ws.counters);
  } else {
    hipLaunchKernelGGL((validate_tiles_kernel<false, true>), dim3(persistent_grid<false, true>()), dim3(kWave), 0, s,
                       sc, qa, qb, n_edges, ws.n_states, ws.offsets, ws.flags, ws.counters);
  }
  hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)g256), dim3(256), 0, s, ws.flags, n_edges, out_valid,
                     ws.counters);
  return hipGetLastError();
}

}  // namespace mrpop
