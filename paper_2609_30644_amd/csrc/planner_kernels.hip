// Planner kernels: sampling, cost-bounded nearest neighbour, the dRRT
// extension oracle, tree insertion, connection selection, path extraction,
// and per-arm roadmap growth (sample, neighbour pairs, adjacency, BFS).
//
// The planner runs in bulk-synchronous rounds of P candidates (the paper runs
// hundreds of iterations at once, one per block; Alg. 2).  Every random
// number comes from a counter-based SplitMix64 stream keyed by (seed,
// purpose, round, candidate), so a round's result does not depend on how the
// work is scheduled.
#include <algorithm>

#include "device_common.h"
#include "planner.h"

namespace mrpop {

// ---------------------------------------------------------------------------
// Counter-based random numbers (SplitMix64; Steele, Lea and Flood 2014)
// ---------------------------------------------------------------------------

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

__host__ __device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__host__ __device__ inline uint64_t stream_key(uint64_t seed, uint64_t a, uint64_t b, uint64_t c) {
  uint64_t k = mix64(seed + kGamma * (a + 1));
  k = mix64(k + kGamma * (b + 1));
  return mix64(k + kGamma * (c + 1));
}

// i-th uniform of a stream in [0, 1): top 24 bits (exact in single precision)
__device__ inline float uniform01(uint64_t key, uint64_t i) {
  return (float)(mix64(key + kGamma * (i + 1)) >> 40) * (1.0f / 16777216.0f);
}

// Standard normal pair p of a stream (Box-Muller on uniforms 2p, 2p+1).
__device__ inline float2 normal_pair(uint64_t key, int p) {
  const float u1 = 1.0f - uniform01(key, 2 * p), u2 = uniform01(key, 2 * p + 1);
  const float rad = sqrtf(-2.0f * logf(u1));
  float s, c;
  sincosf(6.283185307179586f * u2, &s, &c);
  return make_float2(rad * c, rad * s);
}

__device__ inline float normal_at(uint64_t key, int j) {
  const float2 z = normal_pair(key, j >> 1);
  return (j & 1) ? z.y : z.x;
}

// ---------------------------------------------------------------------------
// a2: candidate sampling
// ---------------------------------------------------------------------------

// One wavefront per candidate, one lane per dimension (D <= 2 x 64 handled
// in two strided passes).  c_best = +inf: q_rand uniform in the joint box and
// c_rand = +inf.  Otherwise q_rand is the informed sample (prolate
// hyperspheroid with foci q_s, q_g and transverse diameter c_best; a uniform
// point of the unit D-ball from D normals scaled by u^(1/D), stretched along
// the focal axis, reflected onto it, centred, clamped to the limits) and
// c_rand ~ U[|q_rand - root|, c_best].
constexpr int kSampleWaves = 4;
constexpr int kSamplePer = kMaxDof / kWave + 1;  // dimensions per lane

__device__ __forceinline__ float wave_sum(float v) {
  for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

// Candidate i by one wavefront (lane: its lane index).
__device__ __forceinline__ void sample_one(const SampleArgs &a, int i, int lane) {
  const int D = a.dim;
  float *q = a.out_q + (int64_t)i * D;
  if (!(a.c_best < INFINITY)) {
    const uint64_t k = stream_key(a.seed, kPurposeQ, a.round, a.first + i);
    for (int j = lane; j < D; j += kWave) q[j] = fmaf(uniform01(k, j), a.hi[j] - a.lo[j], a.lo[j]);
    if (a.out_c && lane == 0) a.out_c[i] = INFINITY;
    return;
  }
  const uint64_t k = stream_key(a.seed, kPurposeBall, a.round, a.first + i);
  float cmin2 = 0.f;
  for (int j = lane; j < D; j += kWave) {
    const float d = a.qg[j] - a.qs[j];
    cmin2 = fmaf(d, d, cmin2);
  }
  cmin2 = wave_sum(cmin2);
  const float cmin = sqrtf(cmin2);
  const float r1 = 0.5f * a.c_best;
  const float rr = a.c_best * a.c_best - cmin2;
  const float r2 = rr > 0.f ? 0.5f * sqrtf(rr) : 0.f;
  // |z|^2, and v . (L z) with v = e_1 - (q_g - q_s) / c_min
  float z[kSamplePer], v[kSamplePer];
  float n2 = 0.f, vy = 0.f, vv = 0.f;
#pragma unroll
  for (int t = 0; t < kSamplePer; ++t) {
    const int j = lane + t * kWave;
    z[t] = 0.f;
    v[t] = 0.f;
    if (j < D) {
      z[t] = normal_at(k, j);
      n2 = fmaf(z[t], z[t], n2);
      const float a1 = cmin > 0.f ? (a.qg[j] - a.qs[j]) / cmin : (j == 0 ? 1.f : 0.f);
      v[t] = (j == 0 ? 1.f : 0.f) - a1;
      vv = fmaf(v[t], v[t], vv);
      vy = fmaf(v[t], z[t] * (j == 0 ? r1 : r2), vy);
    }
  }
  n2 = wave_sum(n2);
  vv = wave_sum(vv);
  vy = wave_sum(vy);
  const int pairs = (D + 1) / 2;
  const float scale = powf(uniform01(k, 2 * pairs), 1.0f / (float)D) / sqrtf(n2);
  const float refl = vv > 1e-30f ? 2.f * scale * vy / vv : 0.f;
  // q = centre + H (scale L z), clamped
  float lb2 = 0.f;
#pragma unroll
  for (int t = 0; t < kSamplePer; ++t) {
    const int j = lane + t * kWave;
    if (j < D) {
      const float y = scale * z[t] * (j == 0 ? r1 : r2);
      float x = 0.5f * (a.qs[j] + a.qg[j]) + (vv > 1e-30f ? y - v[t] * refl : y);
      x = fminf(fmaxf(x, a.lo[j]), a.hi[j]);
      q[j] = x;
      const float d = x - a.root[j * a.root_stride];
      lb2 = fmaf(d, d, lb2);
    }
  }
  lb2 = wave_sum(lb2);
  if (a.out_c && lane == 0) {
    const float lb = sqrtf(lb2);
    const float u = uniform01(stream_key(a.seed, kPurposeC, a.round, a.first + i), 0);
    a.out_c[i] = lb < a.c_best ? fmaf(u, a.c_best - lb, lb) : a.c_best;
  }
}

__device__ __forceinline__ void sample_body(const SampleArgs &a, int bx) {
  const int i = bx * kSampleWaves + (int)(threadIdx.x / kWave);
  if (i >= a.n) return;  // whole waves leave together
  sample_one(a, i, (int)(threadIdx.x & (kWave - 1)));
}

// ---------------------------------------------------------------------------
// a3: cost-bounded nearest neighbour (NEAREST of Alg. 2)
// ---------------------------------------------------------------------------

struct Best {
  float d2, g;
  int32_t idx;
};

__device__ __forceinline__ bool better(const Best &a, const Best &b) {
  if (a.idx < 0) return false;
  if (b.idx < 0) return true;
  if (a.d2 != b.d2) return a.d2 < b.d2;
  if (a.g != b.g) return a.g < b.g;
  return a.idx < b.idx;
}

// This thread's best vertex (threads stride over vertices) for the query sq
// under budget c; DC > 0: the dimension, known at compile time.  Squared
// distances are summed over the coordinates in order in either form.
template <int DC>
__device__ __forceinline__ Best nearest_scan(const NearestArgs &a, const float *sq, float c) {
  Best best{INFINITY, INFINITY, -1};
  constexpr int QR = DC > 0 ? DC : 1;
  float q[QR];
  if constexpr (DC > 0) {
#pragma unroll
    for (int j = 0; j < DC; ++j) q[j] = sq[j];
  }
  auto consider = [&](int64_t v, float d2) {
    const float g = a.g ? a.g[v] : 0.f;
    if (!(g + sqrtf(d2) < c)) return;
    const Best cand{d2, g, (int32_t)v};
    if (better(cand, best)) best = cand;
  };
  if constexpr (DC > 0 && DC <= 28) {
    // two vertices per step, both loaded before either is reduced, so that
    // a thread waits on memory once per pair (same per-vertex arithmetic and
    // the same vertex order; larger dimensions keep one, for registers)
    for (int64_t v = threadIdx.x; v < a.n; v += 2 * (int64_t)blockDim.x) {
      const int64_t w = v + blockDim.x;
      const bool has_w = w < a.n;
      const float *p = a.V + v * a.v_stride, *pw = a.V + (has_w ? w : v) * a.v_stride;
      float d2 = 0.f, d2w = 0.f;
#pragma unroll
      for (int j = 0; j < DC; ++j) {
        const float t = q[j] - p[j * a.d_stride], tw = q[j] - pw[j * a.d_stride];
        d2 = fmaf(t, t, d2);
        d2w = fmaf(tw, tw, d2w);
      }
      consider(v, d2);
      if (has_w) consider(w, d2w);
    }
  } else {
    for (int64_t v = threadIdx.x; v < a.n; v += blockDim.x) {
      float d2 = 0.f;
      const float *p = a.V + v * a.v_stride;
      if constexpr (DC > 0) {
#pragma unroll
        for (int j = 0; j < DC; ++j) {
          const float t = q[j] - p[j * a.d_stride];
          d2 = fmaf(t, t, d2);
        }
      } else {
        for (int j = 0; j < a.dim; ++j) {
          const float t = sq[j] - p[j * a.d_stride];
          d2 = fmaf(t, t, d2);
        }
      }
      consider(v, d2);
    }
  }
  return best;
}

// One workgroup per query: threads stride over vertices; admissible when
// g_v + |q - q_v| < c; the least distance wins, ties to the lower cost, then
// the lower index.
__device__ __forceinline__ void nearest_body(const NearestArgs &a, int bx) {
  if (bx >= a.n_queries) return;

  __shared__ float sq[kMaxDof];
  __shared__ Best sb[256 / kWave];
  const int64_t qi = bx;
  const int D = a.dim;
  const float c = a.budgets ? a.budgets[qi] : INFINITY;
  if (!(c > 0.f)) {  // g_v + |q - q_v| >= 0: no vertex is admissible
    if (threadIdx.x == 0) a.out_idx[qi] = -1;
    return;
  }
  for (int j = threadIdx.x; j < D; j += blockDim.x) sq[j] = a.queries[qi * a.q_stride + j];
  __syncthreads();
  Best best;
  switch (D) {  // common dimensions unrolled, with the query in registers
    case 7: best = nearest_scan<7>(a, sq, c); break;
    case 14: best = nearest_scan<14>(a, sq, c); break;
    case 28: best = nearest_scan<28>(a, sq, c); break;
    case 56: best = nearest_scan<56>(a, sq, c); break;
    default: best = nearest_scan<0>(a, sq, c); break;
  }
  for (int d = kWave / 2; d > 0; d >>= 1) {
    Best o;
    o.d2 = __shfl_xor(best.d2, d, kWave);
    o.g = __shfl_xor(best.g, d, kWave);
    o.idx = __shfl_xor(best.idx, d, kWave);
    if (better(o, best)) best = o;
  }
  if ((threadIdx.x & (kWave - 1)) == 0) sb[threadIdx.x / kWave] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    Best b = sb[0];
    for (int w = 1; w < (int)(blockDim.x / kWave); ++w)
      if (better(sb[w], b)) b = sb[w];
    a.out_idx[qi] = b.idx;
  }
}

// ---------------------------------------------------------------------------
// a4: dRRT extension oracle (ORACLE_AOX)
// ---------------------------------------------------------------------------

// One wavefront per candidate.  The arms are searched at the same time, each
// by a group of lanes (64 / R rounded down to a power of two, at least 4):
// the group scans the roadmap neighbours u of the arm's vertex v in q_near.
// Under a finite budget only admissible neighbours count: moving this arm
// alone must keep g_near + |V_u - V_v| < c_rand.  Among them the group keeps
// the one best aligned with the sample direction: largest cosine, ties to the
// lowest neighbour id, so the result does not depend on the order of an
// adjacency row or on how lanes share it; the arm stays if no cosine is
// positive.  If the arms' moves together exceed the budget, moving arms go
// back to staying, least aligned first (ties: the higher arm index first),
// until g_near + |q_new - q_near| < c_rand; the last moving arm always fits
// on its own.  The candidate survives if some arm moves.  |q_new - q_near|^2
// is the sum of the moving arms' |V_u - V_v|^2 (each summed joint by joint)
// in a fixed butterfly order.  Writes the edge to validate (q_near -> q_new);
// dropped candidates get a null edge at q_near.  One wave per candidate (no
// LDS, no barrier).
__device__ __forceinline__ void extend_one(const ExtendArgs &a, int i, int lane) {
  const int D = a.dim, R = a.n_robots;
  const int near = a.near_idx[i];
  float *ea = a.edge_a ? a.edge_a + (int64_t)i * D : nullptr;
  float *eb = a.edge_b ? a.edge_b + (int64_t)i * D : nullptr;
  float *qn = a.q_new + (int64_t)i * D;
  const float *qr = a.q_rand + (int64_t)i * D;
  if (near < 0) {
    if (lane == 0) {
      a.alive[i] = 0;
      a.g_new[i] = INFINITY;
    }
    for (int j = lane; j < D; j += kWave) {
      const float y = a.tree_q[(int64_t)j * a.tree_cap];
      qn[j] = y;
      if (ea) ea[j] = eb[j] = y;
    }
    for (int r = lane; r < R; r += kWave) a.vid_new[(int64_t)r * a.n + i] = -1;
    if (lane == 0 && a.n_codes) a.n_codes[i] = 1;  // a null edge at a tree vertex (finite)
    return;
  }
  const float g_near = a.tree_g[near];
  const float c_rand = a.c_rand ? a.c_rand[i] : INFINITY;
  const bool bounded = c_rand < INFINITY;
  int gs = kWave;  // lanes per arm (MRPOP_MAX_ROBOTS <= 16 arms: at least 4)
  while (gs > 4 && gs * R > kWave) gs >>= 1;
  const int g = lane / gs, sub = lane & (gs - 1);
  // lane r * gs ends with arm r's choice, its cosine and |V_u - V_v|^2
  int best = -1, v = -1;
  float best_cos = 0.f, best_d2 = 0.f;
  if (g < R) {
    const int r = g;
    const int nj = a.nj[r], q0 = a.q_off[r];
    v = a.tree_vid[(int64_t)r * a.tree_cap + near];
    const float *V = a.rm_V + ((int64_t)r * a.rm_cap) * kRmStride;
    const int32_t *rp = a.rm_rowptr + (int64_t)r * (a.rm_cap + 1);
    const int32_t *col = a.rm_col + (int64_t)r * a.rm_col_cap;
    float dir[MRPOP_MAX_JOINTS];
    float dn2 = 0.f;
    for (int j = 0; j < nj; ++j) {
      dir[j] = qr[q0 + j] - V[(int64_t)v * kRmStride + j];
      dn2 = fmaf(dir[j], dir[j], dn2);
    }
    best = v;
    if (dn2 > 0.f) {
      const float dn = sqrtf(dn2);
      const int e0 = rp[v], e1 = min(rp[v + 1], a.rm_col_cap);
      for (int e = e0 + sub; e < e1; e += gs) {
        const int u = col[e];
        float dot = 0.f, en2 = 0.f;
        for (int j = 0; j < nj; ++j) {
          const float ej = V[(int64_t)u * kRmStride + j] - V[(int64_t)v * kRmStride + j];
          dot = fmaf(ej, dir[j], dot);
          en2 = fmaf(ej, ej, en2);
        }
        if (en2 <= 0.f) continue;
        if (bounded && !(g_near + sqrtf(en2) < c_rand)) continue;  // not admissible even alone
        const float cs = dot / (sqrtf(en2) * dn);
        if (cs > best_cos || (cs == best_cos && best != v && u < best)) {
          best_cos = cs;
          best = u;
          best_d2 = en2;
        }
      }
    }
    // reduction within the group (partners lane ^ d stay in the group)
    for (int d = gs / 2; d > 0; d >>= 1) {
      const float oc = __shfl_xor(best_cos, d, kWave);
      const int ob = __shfl_xor(best, d, kWave);
      const float od = __shfl_xor(best_d2, d, kWave);
      const bool o_moves = ob != v, moves = best != v;
      if (o_moves && (!moves || oc > best_cos || (oc == best_cos && ob < best))) {
        best_cos = oc;
        best = ob;
        best_d2 = od;
      }
    }
  }
  // (a group is active or idle as a whole, so the shuffles above read active lanes only)
  // arm r's choice into lane r (every lane takes part in the shuffles)
  const int src = (lane < R ? lane : 0) * gs;
  const int arm_best = __shfl(best, src, kWave), arm_v = __shfl(v, src, kWave);
  const float arm_cos = __shfl(best_cos, src, kWave), arm_d2 = __shfl(best_d2, src, kWave);
  bool moving = lane < R && arm_best != arm_v;
  float total = 0.f;
  for (int pass = 0; pass <= MRPOP_MAX_ROBOTS; ++pass) {  // at most R reverts
    total = wave_sum(moving ? arm_d2 : 0.f);
    if (!bounded || g_near + sqrtf(total) < c_rand) break;
    if (__ballot(moving) == 0ull) break;
    // the least aligned moving arm goes back to staying (ties: higher arm)
    float kc = moving ? arm_cos : INFINITY;
    int ki = moving ? lane : -1;
    for (int d = kWave / 2; d > 0; d >>= 1) {
      const float oc = __shfl_xor(kc, d, kWave);
      const int oi = __shfl_xor(ki, d, kWave);
      if (oc < kc || (oc == kc && oi > ki)) {
        kc = oc;
        ki = oi;
      }
    }
    if (lane == ki) moving = false;
  }
  const bool ok = __ballot(moving) != 0ull;
  const int chosen = moving ? arm_best : arm_v;
  const float gn = g_near + sqrtf(total);
  if (lane == 0) {
    a.g_new[i] = gn;
    a.alive[i] = ok ? 1 : 0;
  }
  if (lane < R) a.vid_new[(int64_t)lane * a.n + i] = chosen;
  // q_new and q_near, composite joint k in lane k % 64 (slot k / 64), loaded
  // in parallel, with the edge's largest joint difference for its state count
  constexpr int kPerLane = kMaxDof / kWave + 1;
  float linf = 0.f;
  bool finite = true;
#pragma unroll
  for (int t = 0; t < kPerLane; ++t) {
    const int k = lane + t * kWave;
    int r = 0;
    while (r + 1 < R && k >= a.q_off[r + 1]) ++r;
    const int br = __shfl(chosen, r, kWave);  // every lane takes part
    if (k < D) {
      const float x = a.rm_V[((int64_t)r * a.rm_cap + br) * kRmStride + (k - a.q_off[r])];
      const float y = a.tree_q[(int64_t)k * a.tree_cap + near];
      const float b = ok ? x : y;
      qn[k] = x;
      if (ea) {
        ea[k] = y;
        eb[k] = b;
      }
      finite = finite && isfinite(y) && isfinite(b);
      linf = fmaxf(linf, fabsf(b - y));
    }
  }
  if (a.n_codes) {
    for (int d = kWave / 2; d > 0; d >>= 1) linf = fmaxf(linf, __shfl_xor(linf, d, kWave));
    const bool all_finite = __ballot(!finite) == 0ull;
    if (lane == 0) a.n_codes[i] = state_count_code(linf, all_finite, a.res);
  }
}

// The extension step alone (mrpop_extend): one wavefront per candidate.
constexpr int kExtendWaves = 4;

__global__ __launch_bounds__(kExtendWaves * kWave) void extend_kernel(ExtendArgs a) {
  const int i = blockIdx.x * kExtendWaves + (int)(threadIdx.x / kWave);
  if (i >= a.n) return;  // whole waves leave together
  extend_one(a, i, (int)(threadIdx.x & (kWave - 1)));
}

hipError_t launch_extend(const ExtendArgs &a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  if (a.dim > kMaxDof || a.n_robots < 1 || a.n_robots > MRPOP_MAX_ROBOTS || (!a.edge_a) != (!a.edge_b))
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(extend_kernel, dim3((unsigned)((a.n + kExtendWaves - 1) / kExtendWaves)),
                     dim3(kExtendWaves * kWave), 0, s, a);
  return hipGetLastError();
}

// Direct mode (no roadmaps): the extension moves from q_near toward q_rand,
// the whole way if it is at most `step` away, else by `step` along the
// segment; a candidate that does not move is dropped, and under a finite
// budget so is one with g_near + |q_new - q_near| >= c_rand (the AO-X rule).
// One wavefront per candidate, one joint per lane; writes the edge to
// validate (q_near -> q_new, or a null edge at q_near when dropped) and its
// state count.  Roadmap fields of `a` are not read.
__device__ __forceinline__ void steer_one(const ExtendArgs &a, int i, int lane) {
  const int D = a.dim;
  const int near = a.near_idx[i];
  float *ea = a.edge_a + (int64_t)i * D, *eb = a.edge_b + (int64_t)i * D, *qn = a.q_new + (int64_t)i * D;
  const float *qr = a.q_rand + (int64_t)i * D;
  for (int r = lane; r < a.n_robots; r += kWave) a.vid_new[(int64_t)r * a.n + i] = 0;
  const int src = near < 0 ? 0 : near;  // dropped candidates: a null edge at the root
  // |q_rand - q_near|^2
  float d2 = 0.f;
  for (int j = lane; j < D; j += kWave) {
    const float t = qr[j] - a.tree_q[(int64_t)j * a.tree_cap + src];
    d2 = fmaf(t, t, d2);
  }
  for (int d = kWave / 2; d > 0; d >>= 1) d2 += __shfl_xor(d2, d, kWave);
  const float dist = sqrtf(d2);
  const bool whole = dist <= a.step;
  const float s = whole ? 1.f : a.step / dist;
  float m2 = 0.f, linf = 0.f;
  bool finite = true;
  for (int j = lane; j < D; j += kWave) {
    const float y = a.tree_q[(int64_t)j * a.tree_cap + src];
    const float x = whole ? qr[j] : fmaf(s, qr[j] - y, y);
    qn[j] = x;
    const float t = x - y;
    m2 = fmaf(t, t, m2);
  }
  for (int d = kWave / 2; d > 0; d >>= 1) m2 += __shfl_xor(m2, d, kWave);
  const float gn = a.tree_g[src] + sqrtf(m2);
  bool ok = near >= 0 && dist > 0.f;
  if (ok && a.c_rand && a.c_rand[i] < INFINITY && !(gn < a.c_rand[i])) ok = false;
  for (int j = lane; j < D; j += kWave) {
    const float y = a.tree_q[(int64_t)j * a.tree_cap + src];
    const float b = ok ? qn[j] : y;
    ea[j] = y;
    eb[j] = b;
    finite = finite && isfinite(y) && isfinite(b);
    linf = fmaxf(linf, fabsf(b - y));
  }
  if (lane == 0) {
    a.g_new[i] = gn;
    a.alive[i] = ok ? 1 : 0;
  }
  if (a.n_codes) {
    for (int d = kWave / 2; d > 0; d >>= 1) linf = fmaxf(linf, __shfl_xor(linf, d, kWave));
    const bool all_finite = __ballot(!finite) == 0ull;
    if (lane == 0) a.n_codes[i] = state_count_code(linf, all_finite, a.res);
  }
}

// ---------------------------------------------------------------------------
// a10: insertion in candidate order; a11: connection edges; a12: selection
// ---------------------------------------------------------------------------

// Connection edge (q_new -> q_conn) of one candidate, one joint per lane; a
// candidate without a connection gets a null edge.

__device__ __forceinline__ void conn_one(const ConnArgs &a, int i, int lane) {
  const int c = a.conn_idx[i];
  float *ea = a.edge_a + (int64_t)i * a.dim, *eb = a.edge_b + (int64_t)i * a.dim;
  float linf = 0.f;
  bool finite = true;
  for (int j = lane; j < a.dim; j += kWave) {
    const float x = a.q_new[(int64_t)i * a.dim + j];
    const float y = c >= 0 ? a.other_q[(int64_t)j * a.tree_cap + c] : x;
    ea[j] = x;
    eb[j] = y;
    finite = finite && isfinite(x) && isfinite(y);
    linf = fmaxf(linf, fabsf(y - x));
  }
  if (a.n_codes) {
    for (int d = kWave / 2; d > 0; d >>= 1) linf = fmaxf(linf, __shfl_xor(linf, d, kWave));
    const bool all_finite = __ballot(!finite) == 0ull;
    if (lane == 0) a.n_codes[i] = state_count_code(linf, all_finite, a.res);
  }
}

// ---------------------------------------------------------------------------
// a round in two kernels: front half (one workgroup per candidate), back half
// (one workgroup)
// ---------------------------------------------------------------------------

// The candidate's sample (wave 0), then its nearest vertex in the extended
// tree.  The sample reaches the other waves through global memory, ordered
// by the workgroup barrier.
__device__ __forceinline__ void sample_near_body(const SampleNearArgs &a, int bx) {
  if (bx >= a.s.n) return;
  if (threadIdx.x < kWave) sample_one(a.s, bx, (int)threadIdx.x);
  __syncthreads();
  nearest_body(a.q, bx);
}

// ---------------------------------------------------------------------------
// ao-dRRT: the cheapest parent and the rewiring proposals of a candidate
// ---------------------------------------------------------------------------

// Element i (0 or 1) of a two-entry array, by a select: a dynamic index into
// a kernel argument or a local struct would place it in scratch memory.
template <class T>
__device__ __forceinline__ T pick(const T (&x)[2], int i) {
  return i ? x[1] : x[0];
}

// Block-wide (256 threads) minimum of (cost, index), ties to the lower index.
struct CostIdx {
  float c;
  int32_t i;
};

__device__ __forceinline__ bool cheaper(const CostIdx &a, const CostIdx &b) {
  if (a.i < 0) return false;
  if (b.i < 0) return true;
  return a.c < b.c || (a.c == b.c && a.i < b.i);
}

__device__ __forceinline__ CostIdx block_min(CostIdx v, CostIdx *s_red) {
  for (int d = kWave / 2; d > 0; d >>= 1) {
    CostIdx o{__shfl_xor(v.c, d, kWave), __shfl_xor(v.i, d, kWave)};
    if (cheaper(o, v)) v = o;
  }
  const int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  __syncthreads();  // s_red may still be read from a previous call
  if ((threadIdx.x & (kWave - 1)) == 0) s_red[w] = v;
  __syncthreads();
  CostIdx b = s_red[0];
  for (int k = 1; k < nw; ++k)
    if (cheaper(s_red[k], b)) b = s_red[k];
  return b;
}

// Whether tree vertex z of the extended tree is a tensor-product neighbour
// of the candidate's composite vertex (every arm stays or moves along a
// roadmap edge, and not all stay): bm holds, per arm, the candidate's vertex
// and its roadmap neighbours as bits.
__device__ __forceinline__ bool tp_neighbour(const uint32_t *bm, const int32_t *vn, const int32_t *tree_vid,
                                             int tree_cap, int R, int rm_cap, int z) {
  bool same = true;
  for (int r = 0; r < R; ++r) {
    const int32_t v = tree_vid[(int64_t)r * tree_cap + z];
    if ((unsigned)v >= (unsigned)rm_cap) return false;
    if (!((bm[r * (kRwMaxRoadmap / 32) + (v >> 5)] >> (v & 31)) & 1u)) return false;
    same = same && v == vn[r];
  }
  return !same;
}

// After the extension (e: the extended tree's fields already chosen), for a
// live candidate i: its parent becomes the tree vertex of least
// g_z + |q_new - q_z| among q_new's tensor-product neighbours in the tree
// (ties: the lower index; q_near is one of them), with g_new, the extension
// edge (parent -> q_new) and its state count replaced; then the tree
// vertices z (other than the parent) with g_new + |q_new - q_z| < g_z become
// proposals, the kRwSlots of largest drop g_z - cost (ties: lower index), each
// with its edge q_new -> q_z for the round's validation.  A dead candidate
// gets no proposals.  Every thread of the workgroup takes part.
__device__ void rewire_front(const ExtendArgs &e, const RewireArgs &rw, int n_tree, int i) {
  __shared__ uint32_t bm[MRPOP_MAX_ROBOTS * (kRwMaxRoadmap / 32)];
  __shared__ int32_t vn[MRPOP_MAX_ROBOTS];
  __shared__ float qn[kMaxDof];
  __shared__ CostIdx s_red[256 / kWave];
  const int D = e.dim, R = e.n_robots, cap = e.tree_cap, words = kRwMaxRoadmap / 32;
  const bool live = e.alive[i] != 0;  // the same in every thread (written before the caller's barrier)
  int n_prop = 0;
  __shared__ int32_t s_pz[kRwSlots];
  __shared__ float s_pc[kRwSlots], s_pl[kRwSlots];
  if (live) {
    for (int r = threadIdx.x; r < R; r += blockDim.x) vn[r] = e.vid_new[(int64_t)r * e.n + i];
    for (int j = threadIdx.x; j < D; j += blockDim.x) qn[j] = e.q_new[(int64_t)i * D + j];
    for (int k = threadIdx.x; k < R * words; k += blockDim.x) bm[k] = 0u;
    __syncthreads();
    for (int r = 0; r < R; ++r) {
      const int v = vn[r];
      const int32_t *rp = e.rm_rowptr + (int64_t)r * (e.rm_cap + 1);
      const int32_t *col = e.rm_col + (int64_t)r * e.rm_col_cap;
      const int e0 = rp[v], e1 = min(rp[v + 1], e.rm_col_cap);
      for (int k = e0 + (int)threadIdx.x; k < e1; k += blockDim.x) {
        const int u = col[k];
        if ((unsigned)u < (unsigned)e.rm_cap) atomicOr(&bm[r * words + (u >> 5)], 1u << (u & 31));
      }
      if (threadIdx.x == 0) atomicOr(&bm[r * words + (v >> 5)], 1u << (v & 31));
    }
    __syncthreads();
    // 1. the cheapest neighbouring parent
    CostIdx best{INFINITY, -1};
    for (int z = threadIdx.x; z < n_tree; z += blockDim.x) {
      if (!tp_neighbour(bm, vn, e.tree_vid, cap, R, e.rm_cap, z)) continue;
      float d2 = 0.f;
      for (int j = 0; j < D; ++j) {
        const float t = qn[j] - e.tree_q[(int64_t)j * cap + z];
        d2 = fmaf(t, t, d2);
      }
      const CostIdx c{e.tree_g[z] + sqrtf(d2), z};
      if (cheaper(c, best)) best = c;
    }
    best = block_min(best, s_red);
    // q_near is a neighbour, so a parent exists (kept as a guard)
    const int par = best.i >= 0 ? best.i : e.near_idx[i];
    float len = 0.f;
    {
      float d2 = 0.f;
      for (int j = 0; j < D; ++j) {
        const float t = qn[j] - e.tree_q[(int64_t)j * cap + par];
        d2 = fmaf(t, t, d2);
      }
      len = sqrtf(d2);
    }
    const float g_new = best.i >= 0 ? best.c : e.tree_g[par] + len;
    // the extension edge from the parent, with its state count (wave 0)
    if (threadIdx.x < kWave) {
      const int lane = (int)threadIdx.x;
      float linf = 0.f;
      bool finite = true;
      for (int j = lane; j < D; j += kWave) {
        const float y = e.tree_q[(int64_t)j * cap + par];
        e.edge_a[(int64_t)i * D + j] = y;
        e.edge_b[(int64_t)i * D + j] = qn[j];
        finite = finite && isfinite(y) && isfinite(qn[j]);
        linf = fmaxf(linf, fabsf(qn[j] - y));
      }
      for (int d = kWave / 2; d > 0; d >>= 1) linf = fmaxf(linf, __shfl_xor(linf, d, kWave));
      const bool all_finite = __ballot(!finite) == 0ull;
      if (lane == 0) {
        if (e.n_codes) e.n_codes[i] = state_count_code(linf, all_finite, e.res);
        // the round's near_idx array is the parent list of the back half
        const_cast<int32_t *>(e.near_idx)[i] = par;
        e.g_new[i] = g_new;
        rw.e_new[i] = len;
      }
    }
    // 2. proposals: every thread keeps its kRwSlots best (largest drop, then
    // lower index), then the block takes the kRwSlots best of all
    float top_d[kRwSlots], top_c[kRwSlots], top_l[kRwSlots];
    int top_z[kRwSlots];
#pragma unroll
    for (int k = 0; k < kRwSlots; ++k) {
      top_d[k] = -INFINITY;
      top_z[k] = -1;
      top_c[k] = top_l[k] = 0.f;
    }
    for (int z = threadIdx.x; z < n_tree; z += blockDim.x) {
      if (z == par || !tp_neighbour(bm, vn, e.tree_vid, cap, R, e.rm_cap, z)) continue;
      float d2 = 0.f;
      for (int j = 0; j < D; ++j) {
        const float t = qn[j] - e.tree_q[(int64_t)j * cap + z];
        d2 = fmaf(t, t, d2);
      }
      const float l = sqrtf(d2), c = g_new + l, gz = e.tree_g[z];
      if (!(c < gz)) continue;
      float dd = gz - c, cc = c, ll = l;
      int zz = z;
#pragma unroll
      for (int k = 0; k < kRwSlots; ++k) {  // insertion into the sorted list (z rises in this thread)
        const bool take = top_z[k] < 0 || dd > top_d[k];
        if (take) {
          const float td = top_d[k], tc = top_c[k], tl = top_l[k];
          const int tz = top_z[k];
          top_d[k] = dd; top_c[k] = cc; top_l[k] = ll; top_z[k] = zz;
          dd = td; cc = tc; ll = tl; zz = tz;
        }
      }
    }
    int head = 0;  // this thread's next unclaimed entry
    for (int k = 0; k < kRwSlots; ++k) {
      // this thread's entry `head` (selected without a dynamic index, which
      // would put the lists in scratch memory)
      float hd = 0.f, hc = 0.f, hl = 0.f;
      int hz = -1;
#pragma unroll
      for (int u = 0; u < kRwSlots; ++u)
        if (u == head) {
          hd = top_d[u];
          hc = top_c[u];
          hl = top_l[u];
          hz = top_z[u];
        }
      // the block's largest remaining drop: minimum of (-drop, index)
      const CostIdx mine{hz >= 0 ? -hd : INFINITY, hz};
      const CostIdx b = block_min(mine, s_red);
      if (b.i < 0) break;
      if (hz >= 0 && hz == b.i) {  // the owner (indices are unique)
        s_pz[k] = hz;
        s_pc[k] = hc;
        s_pl[k] = hl;
        ++head;
      }
      ++n_prop;
    }
    __syncthreads();
  } else if (threadIdx.x == 0) {
    rw.e_new[i] = 0.f;
  }
  // proposal slots, one per wave in turn: edges q_new -> q_z (unused: a null
  // edge with no states)
  const float *q_new = e.q_new + (int64_t)i * D;
  const int lane = (int)(threadIdx.x & (kWave - 1)), wv = (int)(threadIdx.x / kWave);
  for (int k = wv; k < kRwSlots; k += (int)(blockDim.x / kWave)) {
    const int64_t row = (int64_t)i * kRwSlots + k;
    const int z = k < n_prop ? s_pz[k] : -1;
    float linf = 0.f;
    bool finite = true;
    for (int j = lane; j < D; j += kWave) {
      const float x = q_new[j];
      const float y = z >= 0 ? e.tree_q[(int64_t)j * cap + z] : x;
      rw.edge_a[row * D + j] = x;
      rw.edge_b[row * D + j] = y;
      finite = finite && isfinite(x) && isfinite(y);
      linf = fmaxf(linf, fabsf(y - x));
    }
    for (int d = kWave / 2; d > 0; d >>= 1) linf = fmaxf(linf, __shfl_xor(linf, d, kWave));
    const bool all_finite = __ballot(!finite) == 0ull;
    if (lane == 0) {
      rw.prop_z[row] = z;
      rw.prop_cost[row] = z >= 0 ? s_pc[k] : INFINITY;
      rw.prop_len[row] = z >= 0 ? s_pl[k] : 0.f;
      rw.n_codes[row] = z >= 0 ? state_count_code(linf, all_finite, e.res) : 0;
    }
  }
  __syncthreads();
}

// Sample and nearest vertex; the extension (wave 0); the connection budget
// c_best - g_new; the nearest vertex of the other tree under it; the
// connection edge (wave 0).  Each step's outputs reach the next through
// global memory behind a workgroup barrier.  The connection is searched for
// every live candidate before its extension edge is checked: the other tree
// does not change during the round, so the search gives what it would give
// after the check, and both edges go to one validation.
__device__ __forceinline__ void round_front_body(const RoundFrontArgs &A, int bx) {
  if (bx >= A.sn.s.n) return;
  const SearchState st = *A.ss;  // written by the previous round's back half
  const int ta = st.a, tb = 1 - st.a;
  if (st.stop) {  // the search has ended: null edges at the start root with no states
    const int D = A.e.dim;
    float *ea = A.e.edge_a + (int64_t)bx * D, *eb = A.e.edge_b + (int64_t)bx * D;
    float *ca = A.c.edge_a + (int64_t)bx * D, *cb = A.c.edge_b + (int64_t)bx * D;
    for (int j = threadIdx.x; j < D; j += blockDim.x) {
      const float y = A.t.q[0][(int64_t)j * A.e.tree_cap];
      ea[j] = eb[j] = ca[j] = cb[j] = y;
    }
    if (A.rw.on)
      for (int k = 0; k < kRwSlots; ++k) {
        const int64_t row = (int64_t)bx * kRwSlots + k;
        for (int j = threadIdx.x; j < D; j += blockDim.x)
          A.rw.edge_a[row * D + j] = A.rw.edge_b[row * D + j] = A.t.q[0][(int64_t)j * A.e.tree_cap];
        if (threadIdx.x == 0) {
          A.rw.prop_z[row] = -1;
          A.rw.n_codes[row] = 0;
        }
      }
    if (threadIdx.x == 0) {
      A.e.alive[bx] = 0;
      if (A.e.n_codes) A.e.n_codes[bx] = 0;
      if (A.c.n_codes) A.c.n_codes[bx] = 0;
    }
    return;
  }
  SampleNearArgs sn = A.sn;
  sn.s.root = pick(A.t.q, ta);
  sn.q.V = pick(A.t.q, ta);
  sn.q.g = pick(A.t.g, ta);
  sn.q.n = pick(st.n, ta);
  ExtendArgs e = A.e;
  e.tree_q = pick(A.t.q, ta);
  e.tree_vid = pick(A.t.vid, ta);
  e.tree_g = pick(A.t.g, ta);
  NearestArgs q2 = A.q2;
  q2.V = pick(A.t.q, tb);
  q2.g = pick(A.t.g, tb);
  q2.n = pick(st.n, tb);
  ConnArgs c = A.c;
  c.other_q = pick(A.t.q, tb);
  sample_near_body(sn, bx);
  __syncthreads();
  if (threadIdx.x < kWave) {
    const int lane = (int)threadIdx.x;
    if (e.direct) steer_one(e, bx, lane);
    else extend_one(e, bx, lane);
  }
  __syncthreads();
  if (A.rw.on) rewire_front(e, A.rw, pick(st.n, ta), bx);  // ends with a barrier
  // (extend_one's lane 0, or the rewiring step, wrote alive and g_new)
  if (threadIdx.x == 0)
    A.budget[bx] = !e.alive[bx] ? -1.f : (A.c_best < INFINITY ? A.c_best - e.g_new[bx] : INFINITY);
  __syncthreads();
  nearest_body(q2, bx);
  __syncthreads();
  if (threadIdx.x < kWave) conn_one(c, bx, (int)threadIdx.x);
}

// One workgroup of 1024 threads.  Survivors are placed in candidate order
// (a ballot prefix count per wave, wave totals in LDS, chunk by chunk) at
// n_before + rank while the tree has room; then their rows are copied into
// the tree (SoA), and the cheapest free connection among the inserted
// candidates is reduced over lanes and waves.  Connection states of
// candidates that were not inserted are counted apart (speculative work).
__device__ __forceinline__ void publish_status(const RoundStatus &st, RoundStatus *o, uint32_t seq) {
  o->found = st.found;
  o->cand = st.cand;
  o->a_idx = st.a_idx;
  o->b_idx = st.b_idx;
  o->total = st.total;
  o->inserted = st.inserted;
  o->overflow = st.overflow;
  o->a = st.a;
  o->skipped = st.skipped;
  o->states_ext = st.states_ext;
  o->states_conn = st.states_conn;
  o->states_spec = st.states_spec;
  o->states_rw = st.states_rw;
  o->rewired = st.rewired;
  o->n_after = st.n_after;
  __hip_atomic_store(&o->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

__device__ __forceinline__ void insert_select_body(const InsertSelectArgs &a, int bx) {
  if (bx != 0) return;
  const SearchState ss = *a.ss;
  if (ss.stop) {  // the search has ended: an empty record
    if (threadIdx.x == 0) {
      RoundStatus st{};
      st.cand = st.a_idx = st.b_idx = -1;
      st.total = INFINITY;
      st.a = ss.a;
      st.skipped = 1;
      *a.status = st;
      if (a.status_out) publish_status(st, a.status_out, a.seq);
    }
    return;
  }
  const int ta = ss.a, tb = 1 - ss.a;
  float *const tree_q = pick(a.t.q, ta), *const tree_g = pick(a.t.g, ta);
  int32_t *const tree_vid = pick(a.t.vid, ta), *const tree_parent = pick(a.t.parent, ta);
  const float *const other_q = pick(a.t.q, tb), *const other_g = pick(a.t.g, tb);
  const int n_before = pick(ss.n, ta);
  constexpr int kMaxW = 1024 / kWave;
  __shared__ int32_t s_wsum[kMaxW];
  __shared__ int32_t s_base;
  __shared__ float s_cost[kMaxW];
  __shared__ int32_t s_cand[kMaxW], s_ccand[kMaxW];
  __shared__ unsigned long long s_states[2][kMaxW];
  __shared__ int32_t s_ins[kMaxCandidates];  // tree index of each candidate (-1: not inserted)
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  if (threadIdx.x == 0) s_base = 0;
  const int64_t total_states = (threadIdx.x == 0 && a.counters) ? (int64_t)a.counters[1] : 0;
  // Per candidate, in chunks of the block: every scalar the round needs is
  // loaded first, together with the inputs of its connection's cost (which
  // does not depend on the insertion), so that their latencies overlap; then
  // the ranks of the survivors, their insertion, and the cheapest free
  // connection of an inserted candidate (ties: the lowest candidate).
  float best = INFINITY;
  int bi = -1, bc = -1;
  unsigned long long used = 0, spec = 0;
  __syncthreads();
  for (int i0 = 0; i0 < a.n; i0 += blockDim.x) {
    const int i = i0 + threadIdx.x;
    bool ok = false, conn = false;
    int c = -1, near = -1;
    float g = 0.f, e_new = 0.f, tot = INFINITY;
    unsigned long long ns = 0;
    if (i < a.n) {
      ok = a.alive[i] && a.valid[i];
      c = a.conn_idx[i];
      conn = c >= 0 && a.cvalid[i];
      ns = (unsigned long long)max(a.codes_conn[i], 0);
      g = a.g_new[i];
      near = a.near_idx[i];
      if (a.rw.on) e_new = a.rw.e_new[i];
      if (ok && conn) {
        float d2 = 0.f;
        for (int j = 0; j < a.dim; ++j) {
          const float x = a.q_new[(int64_t)i * a.dim + j] - other_q[(int64_t)j * a.tree_cap + c];
          d2 = fmaf(x, x, d2);
        }
        tot = g + sqrtf(d2) + other_g[c];
      }
    }
    const uint64_t bal = __ballot(ok);
    const int before = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) s_wsum[w] = __popcll(bal);
    __syncthreads();
    int off = 0, chunk = 0;
    for (int k = 0; k < nw; ++k) {
      off += k < w ? s_wsum[k] : 0;
      chunk += s_wsum[k];
    }
    if (i < a.n) {
      const int pos = n_before + s_base + off + before;
      const int32_t t = (ok && pos < a.tree_cap) ? pos : -1;
      a.ins_idx[i] = t;
      s_ins[i] = t;
      if (t >= 0) {
        tree_g[t] = g;
        tree_parent[t] = near;
        if (a.rw.on) pick(a.t.e, ta)[t] = e_new;
      }
      if (t >= 0) used += ns;
      else spec += ns;
      if (t >= 0 && conn && (tot < best || (tot == best && (bi < 0 || i < bi)))) {
        best = tot;
        bi = i;
        bc = c;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) s_base += chunk;
    __syncthreads();
  }
  const int all = s_base;
  const int room = a.tree_cap - n_before;
  const int inserted = all < room ? all : room;
  // rows of the inserted candidates (their tree indices in LDS, behind the
  // barrier); kCopyUnroll elements per thread and step, all loaded before any
  // store (the stores could alias the loads for the compiler, which would
  // otherwise wait on each load in turn)
  constexpr int kCopyUnroll = 8;
  const int64_t n_rows = (int64_t)a.n * a.dim, n_vids = (int64_t)a.n * a.n_robots;
  for (int64_t k0 = threadIdx.x; k0 < n_rows; k0 += kCopyUnroll * (int64_t)blockDim.x) {
    float v[kCopyUnroll];
    int32_t t[kCopyUnroll];
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
      const int64_t k = k0 + (int64_t)u * blockDim.x;
      t[u] = -1;
      if (k < n_rows) {
        t[u] = s_ins[k / a.dim];
        v[u] = a.q_new[k];
      }
    }
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
      const int64_t k = k0 + (int64_t)u * blockDim.x;
      if (t[u] >= 0) tree_q[(k - k / a.dim * a.dim) * a.tree_cap + t[u]] = v[u];
    }
  }
  for (int64_t k0 = threadIdx.x; k0 < n_vids; k0 += kCopyUnroll * (int64_t)blockDim.x) {
    int32_t v[kCopyUnroll], t[kCopyUnroll];
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
      const int64_t k = k0 + (int64_t)u * blockDim.x;
      t[u] = -1;
      if (k < n_vids) {
        t[u] = s_ins[k % a.n];
        v[u] = a.vid_new[k];
      }
    }
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
      const int64_t k = k0 + (int64_t)u * blockDim.x;
      if (t[u] >= 0) tree_vid[(k / a.n) * a.tree_cap + t[u]] = v[u];
    }
  }
  for (int d = kWave / 2; d > 0; d >>= 1) {
    const float oc = __shfl_xor(best, d, kWave);
    const int oi = __shfl_xor(bi, d, kWave), ob = __shfl_xor(bc, d, kWave);
    if (oi >= 0 && (bi < 0 || oc < best || (oc == best && oi < bi))) {
      best = oc;
      bi = oi;
      bc = ob;
    }
    used += __shfl_xor(used, d, kWave);
    spec += __shfl_xor(spec, d, kWave);
  }
  if (lane == 0) {
    s_cost[w] = best;
    s_cand[w] = bi;
    s_ccand[w] = bc;
    s_states[0][w] = used;
    s_states[1][w] = spec;
  }
  // ao-dRRT: the proposals of inserted candidates whose edge is free, the
  // cheapest per target (a 64-bit key: cost bits, then the proposal's place
  // in candidate and slot order) when cheaper than the target's cost
  __shared__ int32_t s_rewired;
  __shared__ unsigned long long s_rw_states;
  if (threadIdx.x == 0) {
    s_rewired = 0;
    s_rw_states = 0ull;
  }
  if (a.rw.on) {
    float *const tree_e = pick(a.t.e, ta);
    const int np = a.n * kRwSlots;
    auto usable = [&](int p) {
      const int z = a.rw.prop_z[p];
      return z >= 0 && z < n_before && a.rw.pvalid[p] && s_ins[p / kRwSlots] >= 0;
    };
    for (int p = threadIdx.x; p < np; p += blockDim.x)
      if (usable(p)) a.rw.key[a.rw.prop_z[p]] = ~0ull;
    __syncthreads();
    for (int p = threadIdx.x; p < np; p += blockDim.x)
      if (usable(p))
        atomicMin((unsigned long long *)&a.rw.key[a.rw.prop_z[p]],
                  ((unsigned long long)__float_as_uint(a.rw.prop_cost[p]) << 32) | (unsigned)p);
    __syncthreads();
    int mine = 0;
    unsigned long long rw_states = 0;
    for (int p = threadIdx.x; p < np; p += blockDim.x) {
      rw_states += (unsigned long long)max(a.rw.n_codes[p], 0);
      if (!usable(p)) continue;
      const int z = a.rw.prop_z[p];
      const float c = a.rw.prop_cost[p];
      const unsigned long long k =
          __hip_atomic_load((unsigned long long *)&a.rw.key[z], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (k == (((unsigned long long)__float_as_uint(c) << 32) | (unsigned)p) && c < tree_g[z]) {
        tree_parent[z] = s_ins[p / kRwSlots];
        tree_g[z] = c;
        tree_e[z] = a.rw.prop_len[p];
        ++mine;
      }
    }
    if (mine) atomicAdd(&s_rewired, mine);
    if (rw_states) atomicAdd(&s_rw_states, rw_states);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float bcost = s_cost[0];
    int bc_i = s_cand[0], bc_c = s_ccand[0];
    unsigned long long su = s_states[0][0], ss_ = s_states[1][0];
    for (int k = 1; k < nw; ++k) {
      if (s_cand[k] >= 0 && (bc_i < 0 || s_cost[k] < bcost || (s_cost[k] == bcost && s_cand[k] < bc_i))) {
        bcost = s_cost[k];
        bc_i = s_cand[k];
        bc_c = s_ccand[k];
      }
      su += s_states[0][k];
      ss_ += s_states[1][k];
    }
    const int n_after = n_before + inserted;
    *pick(a.t.n, ta) = n_after;
    RoundStatus st{};
    st.found = bc_i >= 0 ? 1 : 0;
    st.cand = bc_i;
    st.a_idx = bc_i >= 0 ? s_ins[bc_i] : -1;
    st.b_idx = bc_i >= 0 ? bc_c : -1;
    st.total = bcost;
    st.inserted = inserted;
    st.overflow = all > room ? 1 : 0;
    st.a = ta;
    st.skipped = 0;
    st.states_conn = (int64_t)su;
    st.states_spec = (int64_t)ss_;
    st.states_rw = (int64_t)s_rw_states;
    st.states_ext = total_states - (int64_t)su - (int64_t)ss_ - st.states_rw;
    st.rewired = s_rewired;
    st.n_after = n_after;
    *a.status = st;
    // the next round extends the smaller tree (equal sizes: the same one);
    // a connection or a full tree ends the search
    SearchState nx;
    const int n_other = pick(ss.n, tb);
    nx.n[0] = ta == 0 ? n_after : n_other;
    nx.n[1] = ta == 0 ? n_other : n_after;
    nx.a = n_after > n_other ? tb : ta;
    nx.stop = (st.found || st.overflow) ? 1 : 0;
    *a.ss = nx;
    if (a.status_out) publish_status(st, a.status_out, a.seq);
  }
}

// ao-dRRT: after a round that rewired, every vertex's cost is the sum of
// the edge lengths along its parent chain (one thread per vertex; a chain
// has fewer steps than the tree has vertices).
__device__ __forceinline__ void refresh_body(const RefreshArgs &a, int bx) {
  const RoundStatus st = *a.status;
  if (st.skipped || st.rewired <= 0) return;
  const int n = st.n_after;
  const int v = bx * (int)blockDim.x + (int)threadIdx.x;
  if (v >= n) return;
  const int32_t *parent = pick(a.t.parent, st.a);
  const float *e = pick(a.t.e, st.a);
  float acc = 0.f;
  int u = v;
  for (int k = 0; u > 0 && k < n; ++k) {
    acc += e[u];
    u = parent[u];
  }
  pick(a.t.g, st.a)[v] = acc;
}

// Path: root of tree A -> a_idx, then b_idx -> root of tree B (one thread).
__device__ __forceinline__ void path_body(const PathArgs &a, int bx) {
  if (threadIdx.x != 0 || bx != 0) return;
  int len_a = 0;
  for (int v = a.a_idx; v >= 0 && len_a <= a.cap; v = a.parent_a[v]) ++len_a;
  int len_b = 0;
  for (int v = a.b_idx; v >= 0 && len_b <= a.cap; v = a.parent_b[v]) ++len_b;
  const int len = len_a + len_b;
  *a.out_len = len;
  if (len > a.cap) return;
  const int R = a.n_robots;
  int k = len_a - 1;
  for (int v = a.a_idx; v >= 0; v = a.parent_a[v], --k) {
    for (int j = 0; j < a.dim; ++j) a.out[(int64_t)k * a.dim + j] = a.q_a[(int64_t)j * a.tree_cap + v];
    for (int r = 0; r < R; ++r) a.out_vid[(int64_t)k * R + r] = a.vid_a[(int64_t)r * a.tree_cap + v];
  }
  k = len_a;
  for (int v = a.b_idx; v >= 0; v = a.parent_b[v], ++k) {
    for (int j = 0; j < a.dim; ++j) a.out[(int64_t)k * a.dim + j] = a.q_b[(int64_t)j * a.tree_cap + v];
    for (int r = 0; r < R; ++r) a.out_vid[(int64_t)k * R + r] = a.vid_b[(int64_t)r * a.tree_cap + v];
  }
}

// Seed a tree with its root (q, vertex ids of every arm's start or goal).
__device__ __forceinline__ void tree_root_body(const TreeRootArgs &A, int bx) {
  float *tree_q = A.tree_q, *tree_g = A.tree_g;
  int32_t *tree_vid = A.tree_vid, *tree_parent = A.tree_parent, *tree_n = A.tree_n;
  const int tree_cap = A.tree_cap, dim = A.dim, n_robots = A.n_robots, vid = A.vid;
  const float *q = A.q;
  if (bx != 0) return;

  for (int j = threadIdx.x; j < dim; j += blockDim.x) tree_q[(int64_t)j * tree_cap] = q[j];
  for (int r = threadIdx.x; r < n_robots; r += blockDim.x) tree_vid[(int64_t)r * tree_cap] = vid;
  if (threadIdx.x == 0) {
    tree_g[0] = 0.f;
    tree_parent[0] = -1;
    if (A.tree_e) A.tree_e[0] = 0.f;
    *tree_n = 1;
    if (A.ss) *A.ss = SearchState{0, {1, 1}, 0};
  }
}

// ---------------------------------------------------------------------------
// a13: roadmap growth (per arm)
// ---------------------------------------------------------------------------

// Candidate samples j0 .. j0 + n - 1 of an arm's roadmap stream: uniform in
// the arm's joint limits (uniforms 8 j + d of the stream).
__device__ __forceinline__ void rm_sample_body(const RmSampleArgs &A, int bx) {
  float *out = A.out;
  const int n = A.n, nj = A.nj;
  const float *lo = A.lo, *hi = A.hi;
  const uint64_t key = A.key;
  const int64_t j0 = A.j0;

  const int b = bx * blockDim.x + threadIdx.x;
  if (b >= n) return;
  if (A.skip && *A.skip) {  // an arm already connected: no samples, no states
    if (A.codes) A.codes[b] = 0;
    return;
  }
  bool finite = true;
  for (int d = 0; d < nj; ++d) {
    const float x = fmaf(uniform01(key, (uint64_t)(j0 + b) * 8 + d), hi[d] - lo[d], lo[d]);
    out[(int64_t)b * nj + d] = x;
    finite = finite && isfinite(x);
  }
  if (A.codes) A.codes[b] = state_count_code(0.f, finite, 1.f);
}

// Single workgroup: append the first `need` free candidates (in draw order)
// to the roadmap; writes how many were taken.
__device__ __forceinline__ void rm_accept_body(const RmAcceptArgs &A, int bx) {
  const float *cand = A.cand;
  const uint8_t *valid = A.valid;
  const int n = A.n, nj = A.nj, need = A.need, cap = A.cap;
  float *V = A.V;
  int32_t *n_v = A.n_v, *taken = A.taken, *parent = A.parent;
  if (bx != 0) return;

  __shared__ int32_t wsum[1024 / kWave];
  __shared__ int32_t base;
  if (threadIdx.x == 0) base = 0;
  if (threadIdx.x < 2 && A.zero2) A.zero2[threadIdx.x] = 0;
  const int n_eff = (A.skip && *A.skip) ? 0 : n;  // an arm already connected accepts nothing
  __syncthreads();
  for (int i0 = 0; i0 < n_eff; i0 += blockDim.x) {
    const int i = i0 + threadIdx.x;
    const int ok = (i < n_eff && valid[i]) ? 1 : 0;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const uint64_t bal = __ballot(ok);
    const int before = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[w] = __popcll(bal);
    __syncthreads();
    int off = 0, chunk = 0;
    for (int k = 0; k < (int)(blockDim.x / kWave); ++k) {
      if (k < w) off += wsum[k];
      chunk += wsum[k];
    }
    const int pos = base + off + before;
    if (ok && pos < need && *n_v + pos < cap) {
      for (int d = 0; d < nj; ++d) V[(int64_t)(*n_v + pos) * kRmStride + d] = cand[(int64_t)i * nj + d];
      parent[*n_v + pos] = *n_v + pos;  // a new vertex is its own component
    }
    __syncthreads();
    if (threadIdx.x == 0) base += chunk;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    int t = base < need ? base : need;
    if (*n_v + t > cap) t = cap - *n_v;
    *taken = t;
    *n_v += t;
  }
}

// Pairs (j, i), i in [i0, i1) (i1 lowered to the device's vertex count when
// given), j < i, with |V_i - V_j| <= delta: counted (pair_ids null), or
// written as edge endpoints (qa = V_j, qb = V_i) and ids, compacted with an
// atomic counter updated once per wave.  Their order does not reach any
// result: adjacency is rebuilt as a set and the extension oracle breaks ties
// by vertex id.
__device__ __forceinline__ void rm_pairs_body(const RmPairsArgs &A, int bx) {
  const float *V = A.V;
  const int i0 = A.i0, nj = A.nj, cap = A.cap;
  const int i1 = A.i1_dev ? min(A.i1, *A.i1_dev) : A.i1;
  const float delta = A.delta;
  int32_t *count = A.count, *pair_ids = A.pair_ids;
  float *qa = A.qa, *qb = A.qb;

  const int i = i0 + bx;
  if (i >= i1) return;
  const int lane = threadIdx.x & (kWave - 1);
  static_assert(kRmStride == 8, "roadmap rows are read as two float4");
  const float4 *rows = (const float4 *)V;
  const float4 a0 = rows[(int64_t)i * 2], a1 = rows[(int64_t)i * 2 + 1];
  const float vi[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
  for (int j0 = 0; j0 < i; j0 += blockDim.x) {  // the same trip count in every lane
    const int j = j0 + threadIdx.x;
    bool near = false;
    float vj[8];
    if (j < i) {
      const float4 b0 = rows[(int64_t)j * 2], b1 = rows[(int64_t)j * 2 + 1];
      vj[0] = b0.x; vj[1] = b0.y; vj[2] = b0.z; vj[3] = b0.w;
      vj[4] = b1.x; vj[5] = b1.y; vj[6] = b1.z; vj[7] = b1.w;
      float d2 = 0.f;
#pragma unroll
      for (int d = 0; d < 8; ++d)
        if (d < nj) {
          const float t = vi[d] - vj[d];
          d2 = fmaf(t, t, d2);
        }
      near = sqrtf(d2) <= delta;
    }
    // one counter update per wave: slots in lane order within the wave
    const uint64_t m = __ballot(near);
    if (m == 0ull) continue;
    int base = 0;
    if (lane == 0) base = atomicAdd(count, __popcll(m));
    base = __shfl(base, 0, kWave);
    if (!near) continue;
    const int k = base + __popcll(m & ((1ull << lane) - 1ull));
    if (!pair_ids || k >= cap) continue;  // counting only, or beyond the allotted room
    pair_ids[2 * k] = j;
    pair_ids[2 * k + 1] = i;
    bool finite = true;
    float linf = 0.f;
#pragma unroll
    for (int d = 0; d < 8; ++d)
      if (d < nj) {
        const float x = vj[d], y = vi[d];
        qa[(int64_t)k * nj + d] = x;
        qb[(int64_t)k * nj + d] = y;
        finite = finite && isfinite(x) && isfinite(y);
        linf = fmaxf(linf, fabsf(y - x));
      }
    if (A.codes) A.codes[k] = state_count_code(linf, finite, A.res);
  }
}


// Single workgroup: union-find over the arm's roadmap (parent pointers, a
// vertex's parent never has a larger index, so a component's root is its
// smallest vertex and vertex 0 is always a root).  Merges the components of
// the valid new edges, then writes whether vertex 1 shares vertex 0's
// component.  The pointers are worked on in LDS (at most kUfMax vertices).
constexpr int kUfMax = 32768;

__device__ __forceinline__ int uf_find(int32_t *par, int x) {
  for (;;) {
    const int p = par[x];
    if (p == x) return x;
    const int gp = par[p];
    if (gp != p) par[x] = gp;  // path halving (still an ancestor)
    x = gp;
  }
}

__device__ __forceinline__ void rm_union_body(const RmUnionArgs &A, int bx) {
  if (bx != 0) return;
  __shared__ int32_t par[kUfMax];
  const int nv = A.n_v < kUfMax ? A.n_v : kUfMax;
  for (int v = threadIdx.x; v < nv; v += blockDim.x) par[v] = A.parent[v];
  const int np = *A.n_pairs < A.max_pairs ? *A.n_pairs : A.max_pairs;
  if (A.edges) {  // the valid pairs appended to the edge list, one counter update per wave
    const int lane = threadIdx.x & (kWave - 1);
    for (int k0 = 0; k0 < np; k0 += blockDim.x) {
      const int k = k0 + threadIdx.x;
      const bool v = k < np && A.valid[k];
      const uint64_t m = __ballot(v);
      if (m == 0ull) continue;
      int base = 0;
      if (lane == 0) base = atomicAdd(A.n_edges, __popcll(m));
      base = __shfl(base, 0, kWave);
      if (!v) continue;
      const int e = base + __popcll(m & ((1ull << lane) - 1ull));
      if (e >= A.cap_edges) continue;
      A.edges[2 * e] = A.pair_ids[2 * k];
      A.edges[2 * e + 1] = A.pair_ids[2 * k + 1];
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < np; k += blockDim.x) {
    if (!A.valid[k]) continue;
    int a = A.pair_ids[2 * k], b = A.pair_ids[2 * k + 1];
    if (a >= nv || b >= nv) continue;
    for (;;) {  // hook the larger root under the smaller one
      a = uf_find(par, a);
      b = uf_find(par, b);
      if (a == b) break;
      const int hi = a > b ? a : b, lo = a > b ? b : a;
      if (atomicCAS(&par[hi], hi, lo) == hi) break;
    }
  }
  __syncthreads();
  for (int v = threadIdx.x; v < nv; v += blockDim.x) A.parent[v] = uf_find(par, v);
  if (threadIdx.x == 0) {
    const int32_t c = (nv > 1 && uf_find(par, 1) == uf_find(par, 0)) ? 1 : 0;
    *A.connected = c;
    if (A.connected_out) *A.connected_out = c;
  }
  if (A.cnt && A.cnt_out && threadIdx.x < 16) A.cnt_out[threadIdx.x] = A.cnt[threadIdx.x];
}

// Single workgroup: rebuild the arm's adjacency (CSR) from its edge list
// (degree counts and row cursors with LDS atomics), then breadth-first search
// from vertex 0; writes whether vertex 1 is reached.  The order inside an adjacency row is whatever the atomics give:
// the extension oracle's choice does not depend on it.
__device__ __forceinline__ void rm_csr_bfs_body(const RmBfsArgs &A, int bx) {
  const int32_t *edges = A.edges, *n_edges_p = A.n_edges;
  const int cap_edges = A.cap_edges, n_v = A.n_v, col_cap = A.col_cap;
  int32_t *rowptr = A.rowptr, *col = A.col, *deg = A.deg, *level = A.level, *connected = A.connected;
  if (bx != 0) return;

  __shared__ int32_t wsum[1024 / kWave];
  __shared__ int32_t carry;
  __shared__ int changed, stop;
  // degrees and row cursors in LDS when the roadmap fits (every roadmap the
  // planner builds does: at most kUfMax vertices), else in `deg`
  __shared__ int32_t s_cur[kUfMax];
  if (n_v <= kUfMax) deg = s_cur;
  const int ne = *n_edges_p < cap_edges ? *n_edges_p : cap_edges;
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  for (int v = threadIdx.x; v < n_v; v += blockDim.x) deg[v] = 0;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int e = threadIdx.x; e < ne; e += blockDim.x) {
    atomicAdd(&deg[edges[2 * e]], 1);
    atomicAdd(&deg[edges[2 * e + 1]], 1);
  }
  __syncthreads();
  // exclusive scan of the degrees into rowptr; deg becomes each row's cursor
  for (int v0 = 0; v0 < n_v; v0 += blockDim.x) {
    const int v = v0 + threadIdx.x;
    const int x = v < n_v ? deg[v] : 0;
    int incl = x;
    for (int d = 1; d < kWave; d <<= 1) {
      const int y = __shfl_up(incl, d, kWave);
      if (lane >= d) incl += y;
    }
    if (lane == kWave - 1) wsum[w] = incl;
    __syncthreads();
    int off = carry, chunk = 0;
    for (int k = 0; k < nw; ++k) {
      off += k < w ? wsum[k] : 0;
      chunk += wsum[k];
    }
    if (v < n_v) rowptr[v] = deg[v] = off + incl - x;
    __syncthreads();
    if (threadIdx.x == 0) carry += chunk;
    __syncthreads();
  }
  if (threadIdx.x == 0) rowptr[n_v] = carry;
  for (int e = threadIdx.x; e < ne; e += blockDim.x) {
    const int a = edges[2 * e], b = edges[2 * e + 1];
    const int pa = atomicAdd(&deg[a], 1), pb = atomicAdd(&deg[b], 1);
    if (pa < col_cap) col[pa] = b;
    if (pb < col_cap) col[pb] = a;
  }
  if (!level) return;  // adjacency only
  for (int v = threadIdx.x; v < n_v; v += blockDim.x) level[v] = v == 0 ? 0 : -1;
  __syncthreads();
  for (int depth = 0;; ++depth) {
    if (threadIdx.x == 0) changed = 0;
    __syncthreads();
    for (int v = threadIdx.x; v < n_v; v += blockDim.x) {
      if (level[v] != depth) continue;
      const int e1 = rowptr[v + 1] < col_cap ? rowptr[v + 1] : col_cap;
      for (int e = rowptr[v]; e < e1; ++e) {
        const int u = col[e];
        if (level[u] < 0) {
          level[u] = depth + 1;
          changed = 1;
        }
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) stop = !changed || (n_v > 1 && level[1] >= 0);
    __syncthreads();
    if (stop) break;
  }
  if (threadIdx.x == 0) *connected = (n_v > 1 && level[1] >= 0) ? 1 : 0;
}

// ---------------------------------------------------------------------------
// fill and copy (device or mapped pinned host memory)
// ---------------------------------------------------------------------------

constexpr int kCopyBlocksMax = 1024;

__device__ __forceinline__ void fill_body(const FillArgs &a, int bx) {
  for (int64_t i = (int64_t)bx * 256 + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * 256) a.dst[i] = a.value;
}

__device__ __forceinline__ void copy_body(const CopyArgs &a, int bx) {
  unsigned char *d = (unsigned char *)a.dst;
  const unsigned char *src = (const unsigned char *)a.src;
  for (int64_t i = (int64_t)bx * 256 + threadIdx.x; i < a.bytes; i += (int64_t)gridDim.x * 256) d[i] = src[i];
}

// ---------------------------------------------------------------------------
// entry points: one record, or many records (blockIdx.y) per launch
// ---------------------------------------------------------------------------

// A group of up to kGroupMax records passed by value (kernel arguments).
template <class Args>
struct OpGroup {
  Args a[kGroupMax];
};

#define MRPOP_OP_KERNELS_1(name, Args, threads)                                            \
  constexpr int name##_threads = threads;                                                  \
  __global__ __launch_bounds__(threads) void name##_kernel(Args a) { name##_body(a, blockIdx.x); } \
  __global__ __launch_bounds__(threads) void name##_batch_kernel(const Args *records) {     \
    const Args a = records[blockIdx.y];                                                    \
    name##_body(a, blockIdx.x);                                                            \
  }

#define MRPOP_OP_KERNELS(name, Args, threads)                                              \
  MRPOP_OP_KERNELS_1(name, Args, threads)                                                  \
  static_assert(sizeof(OpGroup<Args>) <= 4096, "group of " #Args " exceeds the kernel argument space"); \
  __global__ __launch_bounds__(threads) void name##_group_kernel(OpGroup<Args> g) {        \
    name##_body(g.a[blockIdx.y], blockIdx.x);                                              \
  }

MRPOP_OP_KERNELS(sample, SampleArgs, kSampleWaves * kWave)
MRPOP_OP_KERNELS(nearest, NearestArgs, 256)
MRPOP_OP_KERNELS(path, PathArgs, 64)
MRPOP_OP_KERNELS(tree_root, TreeRootArgs, 128)
MRPOP_OP_KERNELS(rm_sample, RmSampleArgs, 256)
MRPOP_OP_KERNELS(rm_accept, RmAcceptArgs, 1024)
MRPOP_OP_KERNELS(rm_pairs, RmPairsArgs, 256)
MRPOP_OP_KERNELS(rm_csr_bfs, RmBfsArgs, 1024)
MRPOP_OP_KERNELS(rm_union, RmUnionArgs, 1024)
MRPOP_OP_KERNELS(fill, FillArgs, 256)
MRPOP_OP_KERNELS(copy, CopyArgs, 256)
// (a plan's round steps never form a group of independent records)
MRPOP_OP_KERNELS_1(round_front, RoundFrontArgs, 256)
MRPOP_OP_KERNELS(insert_select, InsertSelectArgs, 1024)
MRPOP_OP_KERNELS(refresh, RefreshArgs, 256)

static int clamp_blocks(int64_t b) { return (int)std::min<int64_t>(std::max<int64_t>(b, 0), 0x7fffffff); }

int op_blocks(Op op, const void *p) {
  switch (op) {
    case Op::Sample: {
      const SampleArgs &a = *(const SampleArgs *)p;
      return clamp_blocks((a.n + kSampleWaves - 1) / kSampleWaves);
    }
    case Op::Nearest: return clamp_blocks(((const NearestArgs *)p)->n_queries);
    case Op::Path: return 1;
    case Op::TreeRoot: return 1;
    case Op::RmSample: return clamp_blocks((((const RmSampleArgs *)p)->n + 255) / 256);
    case Op::RmAccept: return 1;
    case Op::RmPairs: {
      const RmPairsArgs &a = *(const RmPairsArgs *)p;
      return clamp_blocks(a.i1 - a.i0);
    }
    case Op::RmBfs: return 1;
    case Op::RmUnion: return 1;
    case Op::Fill: return (int)std::min<int64_t>((((const FillArgs *)p)->n + 255) / 256, kCopyBlocksMax);
    case Op::Copy: return (int)std::min<int64_t>((((const CopyArgs *)p)->bytes + 255) / 256, kCopyBlocksMax);
    case Op::RoundFront: return clamp_blocks(((const RoundFrontArgs *)p)->sn.s.n);
    case Op::InsertSelect: return 1;
    case Op::Refresh: return clamp_blocks((((const RefreshArgs *)p)->tree_cap + 255) / 256);
    case Op::Validate: return 0;
  }
  return 0;
}

size_t op_args_bytes(Op op) {
  switch (op) {
    case Op::Sample: return sizeof(SampleArgs);
    case Op::Nearest: return sizeof(NearestArgs);
    case Op::Path: return sizeof(PathArgs);
    case Op::TreeRoot: return sizeof(TreeRootArgs);
    case Op::RmSample: return sizeof(RmSampleArgs);
    case Op::RmAccept: return sizeof(RmAcceptArgs);
    case Op::RmPairs: return sizeof(RmPairsArgs);
    case Op::RmBfs: return sizeof(RmBfsArgs);
    case Op::RmUnion: return sizeof(RmUnionArgs);
    case Op::Fill: return sizeof(FillArgs);
    case Op::Copy: return sizeof(CopyArgs);
    case Op::RoundFront: return sizeof(RoundFrontArgs);
    case Op::InsertSelect: return sizeof(InsertSelectArgs);
    case Op::Refresh: return sizeof(RefreshArgs);
    case Op::Validate: return 0;
  }
  return 0;
}

// Argument checks shared by both entry points.
static hipError_t op_check(Op op, const void *p) {
  if (op == Op::Sample && ((const SampleArgs *)p)->dim > kMaxDof) return hipErrorInvalidValue;
  if (op == Op::Nearest && ((const NearestArgs *)p)->dim > kMaxDof) return hipErrorInvalidValue;
  if (op == Op::RoundFront) {
    const RoundFrontArgs &a = *(const RoundFrontArgs *)p;
    const int n = a.sn.s.n;
    if (a.sn.s.dim > kMaxDof || a.sn.q.dim > kMaxDof || a.q2.dim > kMaxDof || a.e.dim > kMaxDof ||
        a.sn.q.n_queries != n || a.e.n != n || a.q2.n_queries != n || a.c.n != n ||
        a.e.near_idx != a.sn.q.out_idx || a.q2.queries != a.e.q_new || a.q2.budgets != a.budget ||
        a.c.conn_idx != a.q2.out_idx || !a.e.edge_a || !a.e.edge_b)
      return hipErrorInvalidValue;
    if (a.rw.on && (a.e.direct || a.e.c_rand || a.sn.q.budgets || a.e.rm_cap > kRwMaxRoadmap ||
                    a.e.n_robots > MRPOP_MAX_ROBOTS || !a.rw.prop_z || !a.rw.prop_cost || !a.rw.prop_len ||
                    !a.rw.edge_a || !a.rw.edge_b || !a.rw.n_codes || !a.rw.e_new))
      return hipErrorInvalidValue;
  }
  return hipSuccess;
}

// block size: the one each kernel was compiled for (MRPOP_OP_KERNELS)
#define MRPOP_OP_CASE(OP, name, Args)                                                               \
  case Op::OP:                                                                                     \
    if (batch)                                                                                     \
      hipLaunchKernelGGL(name##_batch_kernel, dim3((unsigned)grid_x, (unsigned)count), dim3(name##_threads), 0, \
                         s, (const Args *)p);                                                      \
    else                                                                                           \
      hipLaunchKernelGGL(name##_kernel, dim3((unsigned)grid_x), dim3(name##_threads), 0, s, *(const Args *)p); \
    break;

#define MRPOP_GROUP_CASE(OP, name, Args)                                                             \
  case Op::OP: {                                                                                   \
    OpGroup<Args> g;                                                                               \
    for (int i = 0; i < n; ++i) g.a[i] = *(const Args *)recs[i];                                   \
    for (int i = n; i < kGroupMax; ++i) g.a[i] = g.a[0];                                           \
    hipLaunchKernelGGL(name##_group_kernel, dim3((unsigned)grid_x, (unsigned)n), dim3(name##_threads), 0, s, g); \
    break;                                                                                         \
  }

static hipError_t launch_group_any(Op op, const void *const *recs, int n, int grid_x, hipStream_t s) {
  switch (op) {
    MRPOP_GROUP_CASE(Sample, sample, SampleArgs)
    MRPOP_GROUP_CASE(Nearest, nearest, NearestArgs)
    MRPOP_GROUP_CASE(Path, path, PathArgs)
    MRPOP_GROUP_CASE(TreeRoot, tree_root, TreeRootArgs)
    MRPOP_GROUP_CASE(RmSample, rm_sample, RmSampleArgs)
    MRPOP_GROUP_CASE(RmAccept, rm_accept, RmAcceptArgs)
    MRPOP_GROUP_CASE(RmPairs, rm_pairs, RmPairsArgs)
    MRPOP_GROUP_CASE(RmBfs, rm_csr_bfs, RmBfsArgs)
    MRPOP_GROUP_CASE(RmUnion, rm_union, RmUnionArgs)
    MRPOP_GROUP_CASE(Fill, fill, FillArgs)
    MRPOP_GROUP_CASE(Copy, copy, CopyArgs)
    MRPOP_GROUP_CASE(InsertSelect, insert_select, InsertSelectArgs)
    MRPOP_GROUP_CASE(Refresh, refresh, RefreshArgs)
    case Op::RoundFront:
    case Op::Validate: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

static hipError_t launch_any(Op op, const void *p, bool batch, int count, int grid_x, hipStream_t s) {
  switch (op) {
    MRPOP_OP_CASE(Sample, sample, SampleArgs)
    MRPOP_OP_CASE(Nearest, nearest, NearestArgs)
    MRPOP_OP_CASE(Path, path, PathArgs)
    MRPOP_OP_CASE(TreeRoot, tree_root, TreeRootArgs)
    MRPOP_OP_CASE(RmSample, rm_sample, RmSampleArgs)
    MRPOP_OP_CASE(RmAccept, rm_accept, RmAcceptArgs)
    MRPOP_OP_CASE(RmPairs, rm_pairs, RmPairsArgs)
    MRPOP_OP_CASE(RmBfs, rm_csr_bfs, RmBfsArgs)
    MRPOP_OP_CASE(RmUnion, rm_union, RmUnionArgs)
    MRPOP_OP_CASE(Fill, fill, FillArgs)
    MRPOP_OP_CASE(Copy, copy, CopyArgs)
    MRPOP_OP_CASE(RoundFront, round_front, RoundFrontArgs)
    MRPOP_OP_CASE(InsertSelect, insert_select, InsertSelectArgs)
    MRPOP_OP_CASE(Refresh, refresh, RefreshArgs)
    case Op::Validate: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_op(Op op, const void *args, hipStream_t s) {
  const hipError_t c = op_check(op, args);
  if (c != hipSuccess) return c;
  const int g = op_blocks(op, args);
  if (g <= 0) return hipSuccess;
  return launch_any(op, args, false, 1, g, s);
}

hipError_t launch_op_group(Op op, const void *const *args, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (n > kGroupMax || op == Op::Validate || op == Op::RoundFront) return hipErrorInvalidValue;
  int g = 0;
  for (int i = 0; i < n; ++i) {
    const hipError_t c = op_check(op, args[i]);
    if (c != hipSuccess) return c;
    g = std::max(g, op_blocks(op, args[i]));
  }
  if (g <= 0) return hipSuccess;
  return launch_group_any(op, args, n, g, s);
}

hipError_t launch_op_batch(Op op, const void *d_args, int count, int grid_x, hipStream_t s) {
  if (count <= 0 || grid_x <= 0) return hipSuccess;
  if (count > 65535) return hipErrorInvalidValue;
  return launch_any(op, d_args, true, count, grid_x, s);
}

hipError_t launch_sample(const SampleArgs &a, hipStream_t s) { return launch_op(Op::Sample, &a, s); }
hipError_t launch_nearest(const NearestArgs &a, hipStream_t s) {
  if (a.n_queries > 0x7fffffff) return hipErrorInvalidValue;
  return launch_op(Op::Nearest, &a, s);
}
hipError_t launch_path(const PathArgs &a, hipStream_t s) { return launch_op(Op::Path, &a, s); }
hipError_t launch_tree_root(const TreeRootArgs &a, hipStream_t s) { return launch_op(Op::TreeRoot, &a, s); }
hipError_t launch_rm_sample(const RmSampleArgs &a, hipStream_t s) { return launch_op(Op::RmSample, &a, s); }
hipError_t launch_rm_accept(const RmAcceptArgs &a, hipStream_t s) { return launch_op(Op::RmAccept, &a, s); }
hipError_t launch_rm_pairs(const RmPairsArgs &a, hipStream_t s) { return launch_op(Op::RmPairs, &a, s); }
hipError_t launch_rm_csr_bfs(const RmBfsArgs &a, hipStream_t s) { return launch_op(Op::RmBfs, &a, s); }
hipError_t launch_rm_union(const RmUnionArgs &a, hipStream_t s) { return launch_op(Op::RmUnion, &a, s); }
hipError_t launch_fill(const FillArgs &a, hipStream_t s) { return launch_op(Op::Fill, &a, s); }
hipError_t launch_copy(const CopyArgs &a, hipStream_t s) { return launch_op(Op::Copy, &a, s); }

uint64_t roadmap_key(uint64_t seed, uint64_t stream_a, uint64_t stream_b) {
  return stream_key(seed, kPurposeRoadmap, stream_a, stream_b);
}

}  // namespace mrpop
