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

__global__ __launch_bounds__(kSampleWaves * kWave) void sample_kernel(SampleArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int i = blockIdx.x * kSampleWaves + (int)(threadIdx.x / kWave);
  if (i >= a.n) return;  // whole waves leave together
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

hipError_t launch_sample(const SampleArgs &a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  if (a.dim > kMaxDof) return hipErrorInvalidValue;
  hipLaunchKernelGGL(sample_kernel, dim3((unsigned)((a.n + kSampleWaves - 1) / kSampleWaves)),
                     dim3(kSampleWaves * kWave), 0, s, a);
  return hipGetLastError();
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

// One workgroup per query: threads stride over vertices; admissible when
// g_v + |q - q_v| < c; the least distance wins, ties to the lower cost, then
// the lower index.
__global__ __launch_bounds__(256) void nearest_kernel(NearestArgs a) {
  __shared__ float sq[kMaxDof];
  __shared__ Best sb[256 / kWave];
  const int64_t qi = blockIdx.x;
  const int D = a.dim;
  for (int j = threadIdx.x; j < D; j += blockDim.x) sq[j] = a.queries[qi * a.q_stride + j];
  __syncthreads();
  const float c = a.budgets ? a.budgets[qi] : INFINITY;
  Best best{INFINITY, INFINITY, -1};
  for (int64_t v = threadIdx.x; v < a.n; v += blockDim.x) {
    float d2 = 0.f;
    for (int j = 0; j < D; ++j) {
      const float t = sq[j] - a.V[v * a.v_stride + j * a.d_stride];
      d2 = fmaf(t, t, d2);
    }
    const float g = a.g ? a.g[v] : 0.f;
    if (!(g + sqrtf(d2) < c)) continue;
    const Best cand{d2, g, (int32_t)v};
    if (better(cand, best)) best = cand;
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

hipError_t launch_nearest(const NearestArgs &a, hipStream_t s) {
  if (a.n_queries <= 0) return hipSuccess;
  if (a.dim > kMaxDof || a.n_queries > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(nearest_kernel, dim3((unsigned)a.n_queries), dim3(256), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// a4: dRRT extension oracle (ORACLE_AOX)
// ---------------------------------------------------------------------------

// One wavefront per candidate.  For every arm,
// the lanes scan the roadmap neighbours of the arm's vertex in q_near and the
// wave keeps the neighbour best aligned with the sample direction: largest
// cosine, ties to the lowest neighbour id, so the result does not depend on
// the order of an adjacency row.  The arm stays if no cosine is positive.
// The candidate survives if some arm moves and, under a finite budget,
// g_near + |q_new - q_near| < c_rand.  Writes the edge to validate
// (q_near -> q_new); dropped candidates get a null edge at q_near.
constexpr int kExtendWaves = 4;

__global__ __launch_bounds__(kExtendWaves * kWave) void extend_kernel(ExtendArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int i = blockIdx.x * kExtendWaves + (int)(threadIdx.x / kWave);
  if (i >= a.n) return;  // whole waves leave together
  const int D = a.dim, R = a.n_robots;
  const int near = a.near_idx[i];
  float *ea = a.edge_a + (int64_t)i * D, *eb = a.edge_b + (int64_t)i * D, *qn = a.q_new + (int64_t)i * D;
  const float *qr = a.q_rand + (int64_t)i * D;
  if (near < 0) {
    if (lane == 0) a.alive[i] = 0;
    for (int j = lane; j < D; j += kWave) ea[j] = eb[j] = qn[j] = a.tree_q[(int64_t)j * a.tree_cap];
    return;
  }
  bool moved = false;
  float dist2 = 0.f;  // identical in every lane
  int my_best = 0;    // lane r keeps arm r's choice
  for (int r = 0; r < R; ++r) {
    const int nj = a.nj[r], q0 = a.q_off[r];
    const int v = a.tree_vid[(int64_t)r * a.tree_cap + near];
    const float *V = a.rm_V + ((int64_t)r * a.rm_cap) * kRmStride;
    const int32_t *rp = a.rm_rowptr + (int64_t)r * (a.rm_cap + 1);
    const int32_t *col = a.rm_col + (int64_t)r * a.rm_col_cap;
    float dir[MRPOP_MAX_JOINTS];
    float dn2 = 0.f;
    for (int j = 0; j < nj; ++j) {
      dir[j] = qr[q0 + j] - V[(int64_t)v * kRmStride + j];
      dn2 = fmaf(dir[j], dir[j], dn2);
    }
    int best = v;
    float best_cos = 0.f;
    if (dn2 > 0.f) {
      const float dn = sqrtf(dn2);
      const int e0 = rp[v], e1 = min(rp[v + 1], a.rm_col_cap);
      for (int e = e0 + lane; e < e1; e += kWave) {
        const int u = col[e];
        float dot = 0.f, en2 = 0.f;
        for (int j = 0; j < nj; ++j) {
          const float ej = V[(int64_t)u * kRmStride + j] - V[(int64_t)v * kRmStride + j];
          dot = fmaf(ej, dir[j], dot);
          en2 = fmaf(ej, ej, en2);
        }
        if (en2 <= 0.f) continue;
        const float cs = dot / (sqrtf(en2) * dn);
        if (cs > best_cos || (cs == best_cos && best != v && u < best)) {
          best_cos = cs;
          best = u;
        }
      }
      for (int d = kWave / 2; d > 0; d >>= 1) {
        const float oc = __shfl_xor(best_cos, d, kWave);
        const int ob = __shfl_xor(best, d, kWave);
        const bool o_moves = ob != v, moves = best != v;
        if (o_moves && (!moves || oc > best_cos || (oc == best_cos && ob < best))) {
          best_cos = oc;
          best = ob;
        }
      }
    }
    moved = moved || best != v;
    if (lane == r) my_best = best;
    for (int j = 0; j < nj; ++j) {
      const float x = V[(int64_t)best * kRmStride + j];
      const float y = a.tree_q[(int64_t)(q0 + j) * a.tree_cap + near];
      dist2 = fmaf(x - y, x - y, dist2);
    }
  }
  const float g = a.tree_g[near] + sqrtf(dist2);
  bool ok = moved;
  if (a.c_rand && a.c_rand[i] < INFINITY && !(g < a.c_rand[i])) ok = false;
  if (lane == 0) {
    a.g_new[i] = g;
    a.alive[i] = ok ? 1 : 0;
  }
  // outputs, one joint per lane (at most 7 joints per arm)
  for (int r = 0; r < R; ++r) {
    const int best = __shfl(my_best, r, kWave);
    const int nj = a.nj[r], q0 = a.q_off[r];
    if (lane == 0) a.vid_new[(int64_t)r * a.n + i] = best;
    if (lane < nj) {
      const float x = a.rm_V[((int64_t)r * a.rm_cap + best) * kRmStride + lane];
      const float y = a.tree_q[(int64_t)(q0 + lane) * a.tree_cap + near];
      qn[q0 + lane] = x;
      ea[q0 + lane] = y;
      eb[q0 + lane] = ok ? x : y;
    }
  }
}

hipError_t launch_extend(const ExtendArgs &a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(extend_kernel, dim3((unsigned)((a.n + kExtendWaves - 1) / kExtendWaves)),
                     dim3(kExtendWaves * kWave), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// a10: insertion in candidate order; a11: connection edges; a12: selection
// ---------------------------------------------------------------------------

// Single workgroup: exclusive scan over surviving candidates (alive and
// edge-valid) in index order; appends them to the tree (SoA) up to its
// capacity; writes each candidate's tree index (-1 if not inserted) and the
// connection budget c_best - g_new (-1 if not inserted, so no vertex is
// admissible).
__global__ __launch_bounds__(1024) void insert_kernel(InsertArgs a) {
  __shared__ int32_t wsum[1024 / kWave];
  __shared__ int32_t base;
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  for (int i0 = 0; i0 < a.n; i0 += blockDim.x) {
    const int i = i0 + threadIdx.x;
    const int ok = (i < a.n && a.alive[i] && a.valid[i]) ? 1 : 0;
    // block exclusive scan of ok
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const uint64_t bal = __ballot(ok);
    const int before = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[w] = __popcll(bal);
    __syncthreads();
    int off = 0;
    for (int k = 0; k < w; ++k) off += wsum[k];
    int chunk = 0;
    for (int k = 0; k < (int)(blockDim.x / kWave); ++k) chunk += wsum[k];
    const int pos = base + off + before;
    if (i < a.n) {
      int32_t t = -1;
      if (ok && *a.tree_n + pos < a.tree_cap) {
        t = *a.tree_n + pos;
        for (int j = 0; j < a.dim; ++j) a.tree_q[(int64_t)j * a.tree_cap + t] = a.q_new[(int64_t)i * a.dim + j];
        for (int r = 0; r < a.n_robots; ++r)
          a.tree_vid[(int64_t)r * a.tree_cap + t] = a.vid_new[(int64_t)r * a.n + i];
        a.tree_g[t] = a.g_new[i];
        a.tree_parent[t] = a.near_idx[i];
      }
      a.ins_idx[i] = t;
      a.budget[i] = t < 0 ? -1.f : (a.c_best < INFINITY ? a.c_best - a.g_new[i] : INFINITY);
    }
    __syncthreads();
    if (threadIdx.x == 0) base += chunk;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int room = a.tree_cap - *a.tree_n;
    const int ins = base < room ? base : room;
    a.status->inserted = ins;
    a.status->overflow = base > room ? 1 : 0;
    *a.tree_n += ins;
  }
}

hipError_t launch_insert(const InsertArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(insert_kernel, dim3(1), dim3(1024), 0, s, a);
  return hipGetLastError();
}

// Connection edges (q_new -> q_conn); candidates without a connection get a
// null edge.
__global__ __launch_bounds__(256) void conn_edges_kernel(ConnArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int c = a.conn_idx[i];
  float *ea = a.edge_a + (int64_t)i * a.dim, *eb = a.edge_b + (int64_t)i * a.dim;
  for (int j = 0; j < a.dim; ++j) {
    const float x = a.q_new[(int64_t)i * a.dim + j];
    ea[j] = x;
    eb[j] = c >= 0 ? a.other_q[(int64_t)j * a.tree_cap + c] : x;
  }
}

hipError_t launch_conn_edges(const ConnArgs &a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(conn_edges_kernel, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

// Single workgroup: among inserted candidates whose connection edge is free,
// the least total cost g_new + |q_new - q_conn| + g_conn (ties: lowest
// candidate index).
__global__ __launch_bounds__(256) void select_kernel(SelectArgs a) {
  __shared__ float sc[256];
  __shared__ int si[256];
  float best = INFINITY;
  int bi = -1;
  for (int i = threadIdx.x; i < a.n; i += blockDim.x) {
    const int c = a.conn_idx[i];
    if (a.ins_idx[i] < 0 || c < 0 || !a.cvalid[i]) continue;
    float d2 = 0.f;
    for (int j = 0; j < a.dim; ++j) {
      const float t = a.q_new[(int64_t)i * a.dim + j] - a.other_q[(int64_t)j * a.tree_cap + c];
      d2 = fmaf(t, t, d2);
    }
    const float tot = a.g_new[i] + sqrtf(d2) + a.other_g[c];
    if (tot < best || (tot == best && (bi < 0 || i < bi))) {
      best = tot;
      bi = i;
    }
  }
  sc[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int t = 1; t < (int)blockDim.x; ++t)
      if (si[t] >= 0 && (si[0] < 0 || sc[t] < sc[0] || (sc[t] == sc[0] && si[t] < si[0]))) {
        sc[0] = sc[t];
        si[0] = si[t];
      }
    a.status->found = si[0] >= 0 ? 1 : 0;
    a.status->cand = si[0];
    a.status->a_idx = si[0] >= 0 ? a.ins_idx[si[0]] : -1;
    a.status->b_idx = si[0] >= 0 ? a.conn_idx[si[0]] : -1;
    a.status->total = sc[0];
    a.status->states_ext = a.states_ext ? (int64_t)a.states_ext[1] : 0;
    a.status->states_conn = a.states_conn ? (int64_t)a.states_conn[1] : 0;
  }
}

hipError_t launch_select(const SelectArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(select_kernel, dim3(1), dim3(256), 0, s, a);
  return hipGetLastError();
}

// Path: root of tree A -> a_idx, then b_idx -> root of tree B (one thread).
__global__ void path_kernel(PathArgs a) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int len_a = 0;
  for (int v = a.a_idx; v >= 0 && len_a <= a.cap; v = a.parent_a[v]) ++len_a;
  int len_b = 0;
  for (int v = a.b_idx; v >= 0 && len_b <= a.cap; v = a.parent_b[v]) ++len_b;
  const int len = len_a + len_b;
  *a.out_len = len;
  if (len > a.cap) return;
  int k = len_a - 1;
  for (int v = a.a_idx; v >= 0; v = a.parent_a[v], --k)
    for (int j = 0; j < a.dim; ++j) a.out[(int64_t)k * a.dim + j] = a.q_a[(int64_t)j * a.tree_cap + v];
  k = len_a;
  for (int v = a.b_idx; v >= 0; v = a.parent_b[v], ++k)
    for (int j = 0; j < a.dim; ++j) a.out[(int64_t)k * a.dim + j] = a.q_b[(int64_t)j * a.tree_cap + v];
}

hipError_t launch_path(const PathArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(path_kernel, dim3(1), dim3(64), 0, s, a);
  return hipGetLastError();
}

// Seed a tree with its root (q, vertex ids of every arm's start or goal).
__global__ void tree_root_kernel(float *tree_q, int32_t *tree_vid, float *tree_g, int32_t *tree_parent, int32_t *tree_n,
                                 int tree_cap, const float *q, int dim, int n_robots, int vid) {
  for (int j = threadIdx.x; j < dim; j += blockDim.x) tree_q[(int64_t)j * tree_cap] = q[j];
  for (int r = threadIdx.x; r < n_robots; r += blockDim.x) tree_vid[(int64_t)r * tree_cap] = vid;
  if (threadIdx.x == 0) {
    tree_g[0] = 0.f;
    tree_parent[0] = -1;
    *tree_n = 1;
  }
}

hipError_t launch_tree_root(float *tree_q, int32_t *tree_vid, float *tree_g, int32_t *tree_parent, int32_t *tree_n,
                            int tree_cap, const float *q, int dim, int n_robots, int vid, hipStream_t s) {
  hipLaunchKernelGGL(tree_root_kernel, dim3(1), dim3(128), 0, s, tree_q, tree_vid, tree_g, tree_parent, tree_n,
                     tree_cap, q, dim, n_robots, vid);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// a13: roadmap growth (per arm)
// ---------------------------------------------------------------------------

// Candidate samples j0 .. j0 + n - 1 of an arm's roadmap stream: uniform in
// the arm's joint limits (uniforms 8 j + d of the stream).
__global__ __launch_bounds__(256) void rm_sample_kernel(float *out, int n, int nj, const float *lo, const float *hi,
                                                        uint64_t key, int64_t j0) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  for (int d = 0; d < nj; ++d)
    out[(int64_t)b * nj + d] = fmaf(uniform01(key, (uint64_t)(j0 + b) * 8 + d), hi[d] - lo[d], lo[d]);
}

hipError_t launch_rm_sample(float *out, int n, int nj, const float *lo, const float *hi, uint64_t seed,
                            uint64_t stream_a, uint64_t stream_b, int64_t j0, hipStream_t s) {
  const uint64_t key = stream_key(seed, kPurposeRoadmap, stream_a, stream_b);
  hipLaunchKernelGGL(rm_sample_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, n, nj, lo, hi, key,
                     j0);
  return hipGetLastError();
}

// Single workgroup: append the first `need` free candidates (in draw order)
// to the roadmap; writes how many were taken.
__global__ __launch_bounds__(1024) void rm_accept_kernel(const float *cand, const uint8_t *valid, int n, int nj,
                                                         int need, float *V, int32_t *n_v, int cap, int32_t *taken) {
  __shared__ int32_t wsum[1024 / kWave];
  __shared__ int32_t base;
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  for (int i0 = 0; i0 < n; i0 += blockDim.x) {
    const int i = i0 + threadIdx.x;
    const int ok = (i < n && valid[i]) ? 1 : 0;
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
    if (ok && pos < need && *n_v + pos < cap)
      for (int d = 0; d < nj; ++d) V[(int64_t)(*n_v + pos) * kRmStride + d] = cand[(int64_t)i * nj + d];
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

hipError_t launch_rm_accept(const float *cand, const uint8_t *valid, int n, int nj, int need, float *V, int32_t *n_v,
                            int cap, int32_t *taken, hipStream_t s) {
  hipLaunchKernelGGL(rm_accept_kernel, dim3(1), dim3(1024), 0, s, cand, valid, n, nj, need, V, n_v, cap, taken);
  return hipGetLastError();
}

// Pairs (j, i), i in [i0, i1), j < i, with |V_i - V_j| <= delta: written as
// edge endpoints (qa = V_j, qb = V_i) and ids, compacted with an atomic
// counter (order is irrelevant: adjacency rows are sorted afterwards).
__global__ __launch_bounds__(256) void rm_pairs_kernel(const float *V, int i0, int i1, int nj, float delta,
                                                       int32_t *count, int cap, int32_t *pair_ids, float *qa,
                                                       float *qb) {
  const int i = i0 + blockIdx.x;
  if (i >= i1) return;
  for (int j = threadIdx.x; j < i; j += blockDim.x) {
    float d2 = 0.f;
    for (int d = 0; d < nj; ++d) {
      const float t = V[(int64_t)i * kRmStride + d] - V[(int64_t)j * kRmStride + d];
      d2 = fmaf(t, t, d2);
    }
    if (!(sqrtf(d2) <= delta)) continue;
    const int k = atomicAdd(count, 1);
    if (k >= cap) continue;
    pair_ids[2 * k] = j;
    pair_ids[2 * k + 1] = i;
    for (int d = 0; d < nj; ++d) {
      qa[(int64_t)k * nj + d] = V[(int64_t)j * kRmStride + d];
      qb[(int64_t)k * nj + d] = V[(int64_t)i * kRmStride + d];
    }
  }
}

hipError_t launch_rm_pairs(const float *V, int i0, int i1, int nj, float delta, int32_t *count, int cap,
                           int32_t *pair_ids, float *qa, float *qb, hipStream_t s) {
  if (i1 <= i0) return hipSuccess;
  hipLaunchKernelGGL(rm_pairs_kernel, dim3((unsigned)(i1 - i0)), dim3(256), 0, s, V, i0, i1, nj, delta, count, cap,
                     pair_ids, qa, qb);
  return hipGetLastError();
}

// Append the valid pairs to the arm's edge list.
__global__ __launch_bounds__(256) void rm_add_edges_kernel(const int32_t *pair_ids, const uint8_t *valid,
                                                           const int32_t *n_pairs, int cap_pairs, int32_t *edges,
                                                           int32_t *n_edges, int cap_edges) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int np = *n_pairs < cap_pairs ? *n_pairs : cap_pairs;
  if (k >= np || !valid[k]) return;
  const int e = atomicAdd(n_edges, 1);
  if (e >= cap_edges) return;
  edges[2 * e] = pair_ids[2 * k];
  edges[2 * e + 1] = pair_ids[2 * k + 1];
}

hipError_t launch_rm_add_edges(const int32_t *pair_ids, const uint8_t *valid, const int32_t *n_pairs, int max_pairs,
                               int32_t *edges, int32_t *n_edges, int cap_edges, hipStream_t s) {
  if (max_pairs <= 0) return hipSuccess;
  hipLaunchKernelGGL(rm_add_edges_kernel, dim3((unsigned)((max_pairs + 255) / 256)), dim3(256), 0, s, pair_ids, valid,
                     n_pairs, max_pairs, edges, n_edges, cap_edges);
  return hipGetLastError();
}

// Single workgroup: rebuild the arm's adjacency (CSR) from its edge list,
// then breadth-first search from vertex 0; writes whether vertex 1 is
// reached.  The order inside an adjacency row is whatever the atomics give:
// the extension oracle's choice does not depend on it.
__global__ __launch_bounds__(1024) void rm_csr_bfs_kernel(const int32_t *edges, const int32_t *n_edges_p,
                                                          int cap_edges, int n_v, int32_t *rowptr, int32_t *col,
                                                          int col_cap, int32_t *deg, int32_t *level,
                                                          int32_t *connected) {
  __shared__ int32_t wsum[1024 / kWave];
  __shared__ int32_t carry;
  __shared__ int changed, stop;
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

hipError_t launch_rm_csr_bfs(const int32_t *edges, const int32_t *n_edges, int cap_edges, int n_v, int32_t *rowptr,
                             int32_t *col, int col_cap, int32_t *deg, int32_t *level, int32_t *connected,
                             hipStream_t s) {
  hipLaunchKernelGGL(rm_csr_bfs_kernel, dim3(1), dim3(1024), 0, s, edges, n_edges, cap_edges, n_v, rowptr, col,
                     col_cap, deg, level, connected);
  return hipGetLastError();
}

}  // namespace mrpop
