// Geometry of the learned initializer's per-view form: the network's input
// points, its proposals in the world frame, and the scene initialisation
// refined by them.  Not part of the paper's method (its Sec. 3.1 initialises
// planes from monocular depth); every reading here is ours.
//
// The file is compiled without floating-point contraction: the refinement
// turns float64 distances into a choice (the nearest proposal) and both the
// kernels and the checks round every operation on its own, in the order
// written.
#include "initnet.h"
#include "ps_internal.h"

using namespace ps;

namespace {

constexpr int kBlock = 256;
constexpr double kWN = 0.25, kWE = 0.25;   // weights of the set loss's normal and extent terms
constexpr double kRMin = 0.01;              // radius floor of a decoded proposal

// Hamilton rotation matrix of a unit quaternion (w, x, y, z), row-major.
__device__ inline void quat_matrix(double w, double x, double y, double z, double R[9]) {
  R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z);       R[2] = 2.0 * (x * z + w * y);
  R[3] = 2.0 * (x * y + w * z);       R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
  R[6] = 2.0 * (x * z - w * y);       R[7] = 2.0 * (y * z + w * x);       R[8] = 1.0 - 2.0 * (x * x + y * y);
}

// Unit quaternion of a rotation matrix (Shepperd's method: the branch of the
// largest of the trace and the diagonal), normalised.
__device__ inline void matrix_quat(const double m[9], double q[4]) {
  const double tr = m[0] + m[4] + m[8];
  if (tr > 0.0) {
    const double s = sqrt(tr + 1.0) * 2.0;
    q[0] = 0.25 * s; q[1] = (m[7] - m[5]) / s; q[2] = (m[2] - m[6]) / s; q[3] = (m[3] - m[1]) / s;
  } else if (m[0] > m[4] && m[0] > m[8]) {
    const double s = sqrt(1.0 + m[0] - m[4] - m[8]) * 2.0;
    q[0] = (m[7] - m[5]) / s; q[1] = 0.25 * s; q[2] = (m[1] + m[3]) / s; q[3] = (m[2] + m[6]) / s;
  } else if (m[4] > m[8]) {
    const double s = sqrt(1.0 + m[4] - m[0] - m[8]) * 2.0;
    q[0] = (m[2] - m[6]) / s; q[1] = (m[1] + m[3]) / s; q[2] = 0.25 * s; q[3] = (m[5] + m[7]) / s;
  } else {
    const double s = sqrt(1.0 + m[8] - m[0] - m[4]) * 2.0;
    q[0] = (m[3] - m[1]) / s; q[1] = (m[2] + m[6]) / s; q[2] = (m[5] + m[7]) / s; q[3] = 0.25 * s;
  }
  const double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int i = 0; i < 4; ++i) q[i] = q[i] / n;
}

// ------------------------------------------------------------------ input points
// One workgroup per view: the candidate pixels in order, the first N with
// depth > 0 kept (order-preserving compaction), each back-projected to the
// camera frame with its depth scaled by 1 + sigma eps; with fewer than N
// valid candidates the kept points repeat in order.
__global__ __launch_bounds__(kBlock) void view_points_kernel(const float* depth, const ps_camera* cams, int H, int W,
                                                             const int32_t* cand, const float* eps, int n_cand, int N,
                                                             float sigma, float* X, int32_t* n_valid) {
  __shared__ int wave_cnt[kBlock / 64];
  const int v = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const ps_camera cam = cams[v];
  const float* D = depth + (size_t)v * H * W;
  float* Xv = X + (size_t)v * N * 3;
  int filled = 0;
  for (int base = 0; base < n_cand && filled < N; base += kBlock) {
    const int i = base + tid;
    int p = -1;
    float z = 0.f;
    if (i < n_cand) {
      p = cand[(size_t)v * n_cand + i];
      if (p >= 0 && p < H * W) z = D[p];
    }
    const bool ok = p >= 0 && p < H * W && z > 0.f;
    const uint64_t m = ballot(ok);
    if (lane == 0) wave_cnt[wid] = __popcll(m);
    __syncthreads();
    int before = filled;
    for (int w = 0; w < wid; ++w) before += wave_cnt[w];
    int total = 0;
    for (int w = 0; w < kBlock / 64; ++w) total += wave_cnt[w];
    const int slot = before + __popcll(m & ((1ull << lane) - 1ull));
    if (ok && slot < N) {
      const double u = (double)(p % W) + 0.5, vv = (double)(p / W) + 0.5;
      const double zz = (double)z * (1.0 + (double)sigma * (double)eps[(size_t)v * n_cand + i]);
      const double dx = (u - (double)cam.cx) / (double)cam.fx;
      const double dy = (vv - (double)cam.cy) / (double)cam.fy;
      Xv[3 * (size_t)slot] = (float)(dx * zz);
      Xv[3 * (size_t)slot + 1] = (float)(dy * zz);
      Xv[3 * (size_t)slot + 2] = (float)zz;
    }
    filled += total;
    __syncthreads();
  }
  const int kept = filled < N ? filled : N;
  __threadfence_block();
  __syncthreads();
  for (int i = kept + tid; i < N; i += kBlock)
    for (int c = 0; c < 3; ++c) Xv[3 * (size_t)i + c] = kept > 0 ? Xv[3 * (size_t)(i % kept) + c] : 0.f;
  if (tid == 0) n_valid[v] = kept;
}

// ------------------------------------------------------------------ proposals to the world frame
__global__ __launch_bounds__(kBlock) void proposals_world_kernel(const float* out, int B, int P, const ps_camera* cams,
                                                                 const int32_t* view_cam, float* center, float* quat,
                                                                 float* radii, float* conf) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= B * P) return;
  const int b = i / P;
  const float* o = out + (size_t)i * IN_OUT;
  const ps_camera cam = cams[view_cam[b]];
  double R[9], t[3];
  for (int k = 0; k < 9; ++k) R[k] = cam.R[k];
  for (int k = 0; k < 3; ++k) t[k] = cam.t[k];
  // decode (camera frame): center, unit quaternion of o[3..6] + (1, 0, 0, 0),
  // radii softplus(o) + 0.01, confidence sigmoid(logit)
  const double c[3] = {(double)o[0] - t[0], (double)o[1] - t[1], (double)o[2] - t[2]};
  double w = (double)o[3] + 1.0, x = o[4], y = o[5], z = o[6];
  const double qn = sqrt(w * w + x * x + y * y + z * z);
  w = w / qn; x = x / qn; y = y / qn; z = z / qn;
  double Rc[9];
  quat_matrix(w, x, y, z, Rc);
  // world: x_w = R^T (x_c - t), rotation R^T Rc
  double Rw[9];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) Rw[3 * r + k] = (R[r] * Rc[k] + R[3 + r] * Rc[3 + k]) + R[6 + r] * Rc[6 + k];
  for (int r = 0; r < 3; ++r) center[3 * (size_t)i + r] = (float)((R[r] * c[0] + R[3 + r] * c[1]) + R[6 + r] * c[2]);
  double q[4];
  matrix_quat(Rw, q);
  for (int k = 0; k < 4; ++k) quat[4 * (size_t)i + k] = (float)q[k];
  for (int k = 0; k < 4; ++k) {
    const double a = o[7 + k];
    const double sp = a > 30.0 ? a : log1p(exp(a));
    radii[4 * (size_t)i + k] = (float)(sp + kRMin);
  }
  conf[i] = (float)(1.0 / (1.0 + exp(-(double)o[11])));
}

// ------------------------------------------------------------------ refinement
// Descriptors of a plane (the set loss's): unit normal n = R(q/|q|) e_z,
// half-extents a >= b from the mean radii of each axis.
__device__ inline void plane_desc(const float* c, const float* q4, const float* r4, double d[9]) {
  double w = q4[0], x = q4[1], y = q4[2], z = q4[3];
  const double qn = sqrt(w * w + x * x + y * y + z * z);
  w = w / qn; x = x / qn; y = y / qn; z = z / qn;
  d[0] = c[0]; d[1] = c[1]; d[2] = c[2];
  d[3] = 2.0 * (x * z + w * y);
  d[4] = 2.0 * (y * z - w * x);
  d[5] = 1.0 - 2.0 * (x * x + y * y);
  const double ex = 0.5 * ((double)r4[0] + (double)r4[1]), ey = 0.5 * ((double)r4[2] + (double)r4[3]);
  d[6] = ex > ey ? ex : ey;
  d[7] = ex > ey ? ey : ex;
  d[8] = 0.0;
}

struct RefineArgs {
  const float *center, *quat, *radii;
  int K;
  const float *pc, *pq, *pr, *pconf;
  int Q;
  double conf_min, d_max;
  float *out_center, *out_quat;
  int32_t* match;
};

// One thread per initial plane; the proposals pass through LDS in tiles.
__global__ __launch_bounds__(kBlock) void refine_kernel(RefineArgs a) {
  __shared__ double tile[9][kBlock];
  const int k = blockIdx.x * kBlock + threadIdx.x;
  const bool act = k < a.K;
  double dk[9] = {0, 0, 0, 0, 0, 1, 0, 0, 0};
  if (act) plane_desc(a.center + 3 * (size_t)k, a.quat + 4 * (size_t)k, a.radii + 4 * (size_t)k, dk);
  double best = 0.0;
  int bi = -1;
  for (int base = 0; base < a.Q; base += kBlock) {
    const int j = base + threadIdx.x;
    if (j < a.Q) {
      double dj[9];
      plane_desc(a.pc + 3 * (size_t)j, a.pq + 4 * (size_t)j, a.pr + 4 * (size_t)j, dj);
      dj[8] = a.pconf[j];
      for (int c = 0; c < 9; ++c) tile[c][threadIdx.x] = dj[c];
    }
    __syncthreads();
    const int n = min(kBlock, a.Q - base);
    for (int jj = 0; jj < n && act; ++jj) {
      if (!(tile[8][jj] >= a.conf_min)) continue;
      const double d0 = tile[0][jj] - dk[0], d1 = tile[1][jj] - dk[1], d2 = tile[2][jj] - dk[2];
      const double dot = (tile[3][jj] * dk[3] + tile[4][jj] * dk[4]) + tile[5][jj] * dk[5];
      const double da = tile[6][jj] - dk[6], db = tile[7][jj] - dk[7];
      const double d = ((d0 * d0 + d1 * d1) + d2 * d2) + kWN * (1.0 - dot * dot) + kWE * (da * da + db * db);
      if (bi < 0 || d < best) {
        best = d;
        bi = base + jj;
      }
    }
    __syncthreads();
  }
  if (!act) return;
  const bool use = bi >= 0 && best <= a.d_max;
  a.match[k] = use ? bi : -1;
  float* oc = a.out_center + 3 * (size_t)k;
  float* oq = a.out_quat + 4 * (size_t)k;
  if (!use) {
    for (int c = 0; c < 3; ++c) oc[c] = a.center[3 * (size_t)k + c];
    for (int c = 0; c < 4; ++c) oq[c] = a.quat[4 * (size_t)k + c];
    return;
  }
  double dp[9];
  plane_desc(a.pc + 3 * (size_t)bi, a.pq + 4 * (size_t)bi, a.pr + 4 * (size_t)bi, dp);
  // the proposal's supporting plane, its normal turned to the initial side;
  // the center moves onto it along that normal
  const double s = ((dp[3] * dk[3] + dp[4] * dk[4]) + dp[5] * dk[5]) < 0.0 ? -1.0 : 1.0;
  const double n[3] = {s * dp[3], s * dp[4], s * dp[5]};
  const double off = ((dk[0] - dp[0]) * n[0] + (dk[1] - dp[1]) * n[1]) + (dk[2] - dp[2]) * n[2];
  for (int c = 0; c < 3; ++c) oc[c] = (float)(dk[c] - off * n[c]);
  // rotation: the smallest one taking the initial normal to n, then the
  // initial frame
  double w = a.quat[4 * (size_t)k], x = a.quat[4 * (size_t)k + 1], y = a.quat[4 * (size_t)k + 2],
         z = a.quat[4 * (size_t)k + 3];
  const double qn = sqrt(w * w + x * x + y * y + z * z);
  w = w / qn; x = x / qn; y = y / qn; z = z / qn;
  double R0[9];
  quat_matrix(w, x, y, z, R0);
  const double v[3] = {dk[4] * n[2] - dk[5] * n[1], dk[5] * n[0] - dk[3] * n[2], dk[3] * n[1] - dk[4] * n[0]};
  const double sn = sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
  const double cs = (dk[3] * n[0] + dk[4] * n[1]) + dk[5] * n[2];
  double A[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  if (sn >= 1e-12) {
    const double u0 = v[0] / sn, u1 = v[1] / sn, u2 = v[2] / sn;
    const double ang = atan2(sn, cs);
    const double si = sin(ang), c1 = 1.0 - cos(ang);
    const double Kx[9] = {0.0, -u2, u1, u2, 0.0, -u0, -u1, u0, 0.0};
    for (int r = 0; r < 3; ++r)
      for (int cc = 0; cc < 3; ++cc) {
        const double kk = (Kx[3 * r] * Kx[cc] + Kx[3 * r + 1] * Kx[3 + cc]) + Kx[3 * r + 2] * Kx[6 + cc];
        A[3 * r + cc] = (A[3 * r + cc] + si * Kx[3 * r + cc]) + c1 * kk;
      }
  }
  double R1[9];
  for (int r = 0; r < 3; ++r)
    for (int cc = 0; cc < 3; ++cc) R1[3 * r + cc] = (A[3 * r] * R0[cc] + A[3 * r + 1] * R0[3 + cc]) + A[3 * r + 2] * R0[6 + cc];
  double q[4];
  matrix_quat(R1, q);
  for (int c = 0; c < 4; ++c) oq[c] = (float)q[c];
}

}  // namespace

extern "C" int initnet_view_points(const float* depth, const ps_camera* cams, int V, int H, int W, const int32_t* cand,
                                   const float* eps, int n_cand, int N, float sigma, float* X, int32_t* n_valid,
                                   void* stream) {
  if (!depth || !cams || !cand || !eps || !X || !n_valid)
    return ps_set_error(PS_ERR_INVALID, "initnet_view_points: null pointer");
  if (V < 1 || H < 1 || W < 1 || n_cand < 1 || N < 1 || (int64_t)H * W >= (int64_t(1) << 31))
    return ps_set_error(PS_ERR_INVALID, "initnet_view_points: bad size");
  hipLaunchKernelGGL(view_points_kernel, dim3(V), dim3(kBlock), 0, (hipStream_t)stream, depth, cams, H, W, cand, eps,
                     n_cand, N, sigma, X, n_valid);
  PS_HIP_CHECK(hipGetLastError());
  return PS_OK;
}

extern "C" int initnet_proposals_to_world(const float* out, int B, int P, const ps_camera* cams,
                                          const int32_t* view_cam, float* center, float* quat, float* radii,
                                          float* conf, void* stream) {
  if (!out || !cams || !view_cam || !center || !quat || !radii || !conf)
    return ps_set_error(PS_ERR_INVALID, "initnet_proposals_to_world: null pointer");
  if (B < 1 || P < 1 || P > IN_PMAX) return ps_set_error(PS_ERR_INVALID, "initnet_proposals_to_world: bad size");
  const int n = B * P;
  hipLaunchKernelGGL(proposals_world_kernel, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, (hipStream_t)stream,
                     out, B, P, cams, view_cam, center, quat, radii, conf);
  PS_HIP_CHECK(hipGetLastError());
  return PS_OK;
}

extern "C" int initnet_refine_planes(const float* center, const float* quat, const float* radii, int K,
                                     const float* p_center, const float* p_quat, const float* p_radii,
                                     const float* p_conf, int Q, double conf_min, double d_max, float* out_center,
                                     float* out_quat, int32_t* match, void* stream) {
  if (!center || !quat || !radii || !out_center || !out_quat || !match ||
      (Q > 0 && (!p_center || !p_quat || !p_radii || !p_conf)))
    return ps_set_error(PS_ERR_INVALID, "initnet_refine_planes: null pointer");
  if (K < 1 || Q < 0) return ps_set_error(PS_ERR_INVALID, "initnet_refine_planes: bad size");
  RefineArgs a{center, quat, radii, K, p_center, p_quat, p_radii, p_conf, Q, conf_min, d_max, out_center, out_quat,
               match};
  hipLaunchKernelGGL(refine_kernel, dim3((K + kBlock - 1) / kBlock), dim3(kBlock), 0, (hipStream_t)stream, a);
  PS_HIP_CHECK(hipGetLastError());
  return PS_OK;
}
