// Device helpers shared by the HIP kernels: rigid frames, the modified
// Denavit-Hartenberg joint step, and small wave utilities.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "mrpop_internal.h"

namespace mrpop {

// Rigid transform [R | t] as three rows.
struct Frame {
  float r00, r01, r02, t0;
  float r10, r11, r12, t1;
  float r20, r21, r22, t2;
};

__device__ __forceinline__ Frame load_frame(const float *__restrict__ p) {
  Frame f;
  f.r00 = p[0]; f.r01 = p[1]; f.r02 = p[2]; f.t0 = p[3];
  f.r10 = p[4]; f.r11 = p[5]; f.r12 = p[6]; f.t1 = p[7];
  f.r20 = p[8]; f.r21 = p[9]; f.r22 = p[10]; f.t2 = p[11];
  return f;
}

// One row of T_{j-1} times the joint transform
//   A = RotX(alpha) TransX(a) RotZ(theta) TransZ(d)
//     = [[c, -s, 0, a], [ca s, ca c, -sa, -sa d], [sa s, sa c, ca, ca d]],
// written with u = R1 ca + R2 sa (the rotated second column).
__device__ __forceinline__ void row_step(float &R0, float &R1, float &R2, float &t, float a, float d, float ca,
                                         float sa, float c, float s) {
  const float u = fmaf(R1, ca, R2 * sa);
  const float n2 = fmaf(R2, ca, -(R1 * sa));
  const float n0 = fmaf(R0, c, u * s);
  const float n1 = fmaf(u, c, -(R0 * s));
  t = fmaf(n2, d, fmaf(R0, a, t));
  R0 = n0;
  R1 = n1;
  R2 = n2;
}

// T_j = T_{j-1} RotX(alpha_{j-1}) TransX(a_{j-1}) RotZ(theta_j) TransZ(d_j)
// (Craig's modified convention).  dh = (a, d, cos alpha, sin alpha).
// The same step from sin(theta_j), cos(theta_j).
__device__ __forceinline__ void joint_step_sc(Frame &T, float4 dh, float s, float c) {
  row_step(T.r00, T.r01, T.r02, T.t0, dh.x, dh.y, dh.z, dh.w, c, s);
  row_step(T.r10, T.r11, T.r12, T.t1, dh.x, dh.y, dh.z, dh.w, c, s);
  row_step(T.r20, T.r21, T.r22, T.t2, dh.x, dh.y, dh.z, dh.w, c, s);
}

__device__ __forceinline__ void joint_step(Frame &T, float4 dh, float theta) {
  float s, c;
  sincosf(theta, &s, &c);
  joint_step_sc(T, dh, s, c);
}

__device__ __forceinline__ float3 apply(const Frame &T, float x, float y, float z) {
  return make_float3(fmaf(T.r00, x, fmaf(T.r01, y, fmaf(T.r02, z, T.t0))),
                     fmaf(T.r10, x, fmaf(T.r11, y, fmaf(T.r12, z, T.t1))),
                     fmaf(T.r20, x, fmaf(T.r21, y, fmaf(T.r22, z, T.t2))));
}

// Squared distance from p to an axis-aligned box: sum of squared per-axis
// excesses max(lo - p, p - hi, 0).
__device__ __forceinline__ float box_dist2(float3 p, float4 lo, float4 hi) {
  const float ex = fmaxf(fmaxf(lo.x - p.x, p.x - hi.x), 0.f);
  const float ey = fmaxf(fmaxf(lo.y - p.y, p.y - hi.y), 0.f);
  const float ez = fmaxf(fmaxf(lo.z - p.z, p.z - hi.z), 0.f);
  return fmaf(ez, ez, fmaf(ey, ey, ex * ex));
}

__device__ __forceinline__ float dist2(float3 a, float4 b) {
  const float dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
  return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
}

__device__ __forceinline__ float dist2(float3 a, float3 b) {
  const float dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
  return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
}

// Read-only scene data viewed through the constant address space: loads with
// wave-uniform addresses then compile to scalar loads (SGPRs, scalar cache)
// instead of vector memory loads, which matters for the obstacle loops.
template <class T>
using cptr = const T __attribute__((address_space(4))) *;

template <class T>
__device__ __forceinline__ cptr<T> as_const(const T *p) {
  return (cptr<T>)p;
}

// float4 element i of a constant-space array (the vector type's copy
// constructor does not bind to constant-space references).
__device__ __forceinline__ float4 ld4(cptr<float4> p, int64_t i) {
  const cptr<float> f = (cptr<float>)p + 4 * i;
  return make_float4(f[0], f[1], f[2], f[3]);
}

__device__ __forceinline__ uint32_t uniform_u32(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Number of states at which an edge is checked (paper, Sec. "Multi-Thread
// Reassignment for Collision Checking": edges are discretised into states),
// from the largest joint difference linf over its endpoints, so that no joint
// moves more than res between states: 1 + ceil(linf / res) in single
// precision with a correctly rounded division, 1 for a null edge.  Negative codes: an
// endpoint is not finite, or the edge would need more than
// MRPOP_MAX_STATES_PER_EDGE states.  Every count of the library is made here.
constexpr int32_t kCodeNonFinite = -1, kCodeTooLong = -2;

__device__ __forceinline__ int32_t state_count_code(float linf, bool finite, float res) {
  if (!finite) return kCodeNonFinite;
  if (linf == 0.f) return 1;
  const float ratio = linf / res;
  if (!(ratio <= (float)(MRPOP_MAX_STATES_PER_EDGE - 1))) return kCodeTooLong;
  return 1 + (int32_t)ceilf(ratio);
}

}  // namespace mrpop
