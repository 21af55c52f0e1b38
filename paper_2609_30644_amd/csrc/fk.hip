// Forward kinematics to world-frame collision spheres.
//
// One lane per (configuration, arm) chain: the lane walks the arm's joints,
// composing modified-DH frames, and writes each link's spheres as soon as the
// link's frame is known, so only the current frame lives in registers.
#include "device_common.h"

namespace mrpop {

__global__ __launch_bounds__(256) void fk_spheres_kernel(SceneDev sc, const float *__restrict__ q, int64_t n_cfg,
                                                         float4 *__restrict__ out) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int R = sc.n_robots;
  if (gid >= n_cfg * R) return;
  const int64_t cfg = gid / R;
  const int r = (int)(gid - cfg * R);
  const int m = sc.model[r];
  const int nj = sc.nj[m];
  const float *qr = q + cfg * sc.dof + sc.q_off[r];
  const int32_t *ls = sc.link_start + m * (kMaxLinks + 1);
  const float4 *fine = sc.fine + (int64_t)m * sc.sph_stride;
  const int32_t *src = sc.fine_src + (int64_t)m * sc.sph_stride;
  float4 *o = out + cfg * sc.total_spheres + sc.s_out[r];
  Frame T = load_frame(sc.base + 12 * r);
  for (int l = 0; l <= nj; ++l) {
    if (l > 0) joint_step(T, sc.dh[m * kMaxJoints + l - 1], qr[l - 1] + sc.theta_off[m * kMaxJoints + l - 1]);
    for (int i = ls[l]; i < ls[l + 1]; ++i) {
      const float4 p = fine[i];
      const float3 w = apply(T, p.x, p.y, p.z);
      o[src[i]] = make_float4(w.x + sc.origin.x, w.y + sc.origin.y, w.z + sc.origin.z, p.w);
    }
  }
}

hipError_t launch_fk_spheres(const SceneDev &sc, const float *q, int64_t n_cfg, float *out, hipStream_t s) {
  const int64_t chains = n_cfg * sc.n_robots;
  const int block = 256;
  const int64_t grid = (chains + block - 1) / block;
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fk_spheres_kernel, dim3((unsigned)grid), dim3(block), 0, s, sc, q, n_cfg, (float4 *)out);
  return hipGetLastError();
}

}  // namespace mrpop
