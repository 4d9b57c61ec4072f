// plane_split / plane_grad_accumulate: the plane-splitting step of the
// fitting loop (Sec. 3.3).  A plane whose average |dL/dr| over its two X
// radii (per-pixel mean loss, averaged over the iterations the plane took
// part in) exceeds the threshold is cut in two across its X extent (halves
// side by side along X), likewise for Y; both gives four children.  Children
// of a plane are consecutive, in plane order: count -> exclusive scan (one
// workgroup) -> write.
#include "ps_internal.h"

using namespace ps;

namespace {

struct SplitArgs {
  const float* center;
  const float* quat;
  const float* radii;
  const float* acc;
  const int* cnt;
  const float* scale;   // per plane, or null for 1
  float thresh;
  int K;
  int* counts;     // [K + 1]
  int* first;      // [K + 1]
  float* oc;
  float* oq;
  float* orad;
  int* parent;
  int* k_out;
};

// The decision is taken in float32 without a division: the average
// (acc+ + acc-) scale / (2 cnt) exceeds thresh.
__device__ inline int split_bits(const SplitArgs& a, int k) {
  const float* g = a.acc + 4 * (size_t)k;
  const float s = a.scale ? a.scale[k] : 1.f;
  const int n = a.cnt[k];
  if (n <= 0) return 0;   // no iteration counted: no average, kept
  const float ct = a.thresh * (float)(2 * n);
  const bool sx = (g[0] + g[1]) * s > ct;
  const bool sy = (g[2] + g[3]) * s > ct;
  return (sx ? 1 : 0) | (sy ? 2 : 0);
}

__global__ void split_count_kernel(SplitArgs a) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < a.K) {
    const int b = split_bits(a, k);
    a.counts[k] = (b & 1 ? 2 : 1) * (b & 2 ? 2 : 1);
  }
}

__global__ __launch_bounds__(1024) void split_scan_kernel(SplitArgs a) {
  __shared__ int lds[40];
  int mx = 0;
  const long long total = block_scan(a.counts, a.first, a.K, lds, mx);
  if (threadIdx.x == 0) *a.k_out = (int)total;
}

__global__ void split_write_kernel(SplitArgs a) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.K) return;
  const int bits = split_bits(a, k);
  // local frame (Eq. 2-3) of the normalised quaternion
  double w = a.quat[4 * k], x = a.quat[4 * k + 1], y = a.quat[4 * k + 2], z = a.quat[4 * k + 3];
  const double qn = sqrt(w * w + x * x + y * y + z * z);
  w /= qn; x /= qn; y /= qn; z /= qn;
  const double vx[3] = {1 - 2 * (y * y + z * z), 2 * (x * y + w * z), 2 * (x * z - w * y)};
  const double vy[3] = {2 * (x * y - w * z), 1 - 2 * (x * x + z * z), 2 * (y * z + w * x)};
  const double rxp = a.radii[4 * k], rxm = a.radii[4 * k + 1];
  const double ryp = a.radii[4 * k + 2], rym = a.radii[4 * k + 3];
  // pieces along each axis: center offset, radius +, radius -
  double xo[2], xr[2][2], yo[2], yr[2][2];
  int nx = 1, ny = 1;
  if (bits & 1) {
    const double m = 0.5 * (rxp - rxm), h = 0.25 * (rxp + rxm);
    xo[0] = m - h; xo[1] = m + h;
    xr[0][0] = xr[0][1] = xr[1][0] = xr[1][1] = h;
    nx = 2;
  } else {
    xo[0] = 0.0; xr[0][0] = rxp; xr[0][1] = rxm;
  }
  if (bits & 2) {
    const double m = 0.5 * (ryp - rym), h = 0.25 * (ryp + rym);
    yo[0] = m - h; yo[1] = m + h;
    yr[0][0] = yr[0][1] = yr[1][0] = yr[1][1] = h;
    ny = 2;
  } else {
    yo[0] = 0.0; yr[0][0] = ryp; yr[0][1] = rym;
  }
  int o = a.first[k];
  for (int i = 0; i < nx; ++i)
    for (int j = 0; j < ny; ++j, ++o) {
      for (int c = 0; c < 3; ++c)
        a.oc[3 * (size_t)o + c] = (float)((double)a.center[3 * k + c] + xo[i] * vx[c] + yo[j] * vy[c]);
      for (int c = 0; c < 4; ++c) a.oq[4 * (size_t)o + c] = a.quat[4 * k + c];
      a.orad[4 * (size_t)o + 0] = (float)xr[i][0];
      a.orad[4 * (size_t)o + 1] = (float)xr[i][1];
      a.orad[4 * (size_t)o + 2] = (float)yr[j][0];
      a.orad[4 * (size_t)o + 3] = (float)yr[j][1];
      a.parent[o] = k;
    }
}

__global__ void grad_acc_kernel(const float4* g, float4* acc, int* cnt, int K) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const float4 x = g[k];
  float4 s = acc[k];
  s.x += fabsf(x.x); s.y += fabsf(x.y); s.z += fabsf(x.z); s.w += fabsf(x.w);
  acc[k] = s;
  if (x.x != 0.f || x.y != 0.f || x.z != 0.f || x.w != 0.f) cnt[k] += 1;
}

}  // namespace

extern "C" int plane_grad_accumulate(const float* g_radii, float* acc, int32_t* cnt, int K, void* stream) {
  if (K < 0 || (K > 0 && (!g_radii || !acc || !cnt)))
    return ps_set_error(PS_ERR_INVALID, "plane_grad_accumulate: bad argument");
  if ((reinterpret_cast<uintptr_t>(g_radii) | reinterpret_cast<uintptr_t>(acc)) & 15)
    return ps_set_error(PS_ERR_INVALID, "plane_grad_accumulate: g_radii and acc must be 16-byte aligned");
  if (K == 0) return PS_OK;
  hipLaunchKernelGGL(grad_acc_kernel, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                     (const float4*)g_radii, (float4*)acc, cnt, K);
  PS_HIP_CHECK(hipGetLastError());
  return PS_OK;
}

extern "C" int plane_split(const float* center, const float* quat, const float* radii, const float* acc,
                           const int32_t* cnt, const float* scale, float thresh, int K, float* out_center,
                           float* out_quat, float* out_radii, int32_t* parent, int32_t* first, int32_t* k_out,
                           int32_t* ws, void* stream) {
  if (K < 1 || !center || !quat || !radii || !acc || !cnt || !out_center || !out_quat || !out_radii || !parent ||
      !first || !k_out || !ws)
    return ps_set_error(PS_ERR_INVALID, "plane_split: bad argument");
  SplitArgs a;
  a.center = center; a.quat = quat; a.radii = radii; a.acc = acc;
  a.cnt = cnt; a.scale = scale;
  a.thresh = thresh;
  a.K = K;
  a.counts = ws; a.first = first;
  a.oc = out_center; a.oq = out_quat; a.orad = out_radii; a.parent = parent; a.k_out = k_out;
  hipStream_t st = (hipStream_t)stream;
  const unsigned g = (unsigned)((K + 255) / 256);
  hipLaunchKernelGGL(split_count_kernel, dim3(g), dim3(256), 0, st, a);
  hipLaunchKernelGGL(split_scan_kernel, dim3(1), dim3(1024), 0, st, a);
  hipLaunchKernelGGL(split_write_kernel, dim3(g), dim3(256), 0, st, a);
  PS_HIP_CHECK(hipGetLastError());
  return PS_OK;
}
