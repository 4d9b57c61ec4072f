// adam_step_planes: bias-corrected Adam on centers, quaternions and radii
// (Sec. 3.3; the paper fixes lr = 1e-3 for all three, beta and epsilon are
// the usual 0.9 / 0.999 / 1e-8).  One thread per scalar parameter; the step
// number is read from device memory so the call can sit in a captured graph.
// Radii are clamped to >= r_min afterwards (they live in R^4_+, Eq. 1).
// Memory-bound: 20 bytes read and 12 written per parameter.
#include "ps_internal.h"

namespace {

struct AdamArgs {
  float* p[3];
  const float* g[3];
  float* m;
  float* v;
  int K;
  const int32_t* step;
  float lr[3];
  float b1, b2, eps, r_min;
};

__global__ __launch_bounds__(256) void adam_kernel(AdamArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = 11 * a.K;
  if (i >= n) return;
  int grp, j;
  if (i < 3 * a.K) { grp = 0; j = i; }
  else if (i < 7 * a.K) { grp = 1; j = i - 3 * a.K; }
  else { grp = 2; j = i - 7 * a.K; }
  float m = a.m[i], v = a.v[i];
  float x = ps::adam_update(a.p[grp][j], a.g[grp][j], m, v, a.lr[grp], a.b1, a.b2, a.eps, a.step[0]);
  a.m[i] = m;
  a.v[i] = v;
  if (grp == 2) x = fmaxf(x, a.r_min);
  a.p[grp][j] = x;
}

}  // namespace

extern "C" int adam_step_planes(float* center, float* quat, float* radii, const float* g_center,
                                const float* g_quat, const float* g_radii, float* m, float* v, int K,
                                const int32_t* step, float lr_center, float lr_quat, float lr_radii,
                                float beta1, float beta2, float eps, float r_min, void* stream) {
  if (K < 0) return ps_set_error(PS_ERR_INVALID, "adam_step_planes: K < 0");
  // an empty plane set (K = 0) may come with null arrays
  if (K > 0 && (!center || !quat || !radii || !g_center || !g_quat || !g_radii || !m || !v || !step))
    return ps_set_error(PS_ERR_INVALID, "adam_step_planes: null pointer");
  if (!(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return ps_set_error(PS_ERR_INVALID, "adam_step_planes: bad beta / eps");
  if (K == 0) return PS_OK;
  AdamArgs a;
  a.p[0] = center; a.p[1] = quat; a.p[2] = radii;
  a.g[0] = g_center; a.g[1] = g_quat; a.g[2] = g_radii;
  a.m = m; a.v = v; a.K = K; a.step = step;
  a.lr[0] = lr_center; a.lr[1] = lr_quat; a.lr[2] = lr_radii;
  a.b1 = beta1; a.b2 = beta2; a.eps = eps; a.r_min = r_min;
  const int n = 11 * K;
  hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, a);
  PS_HIP_CHECK(hipGetLastError());
  return PS_OK;
}

namespace {
// Single-direction radii (the ablation of Sec. 4.3): r^{x+} = r^{x-} is one
// parameter, whose gradient is the sum of the two directions' gradients.
__global__ __launch_bounds__(256) void tie_radii_kernel(float4* g, int K) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  float4 v = g[k];
  const float gx = v.x + v.y, gy = v.z + v.w;
  v.x = gx; v.y = gx; v.z = gy; v.w = gy;
  g[k] = v;
}
}  // namespace

extern "C" int plane_tie_radii(float* g_radii, int K, void* stream) {
  if (K < 0 || (K > 0 && !g_radii)) return ps_set_error(PS_ERR_INVALID, "plane_tie_radii: bad argument");
  if (reinterpret_cast<uintptr_t>(g_radii) & 15)
    return ps_set_error(PS_ERR_INVALID, "plane_tie_radii: g_radii must be 16-byte aligned");
  if (K == 0) return PS_OK;
  hipLaunchKernelGGL(tie_radii_kernel, dim3((K + 255) / 256), dim3(256), 0, (hipStream_t)stream, (float4*)g_radii, K);
  PS_HIP_CHECK(hipGetLastError());
  return PS_OK;
}
