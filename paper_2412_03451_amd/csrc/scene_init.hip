// Scene initialisation (Sec. 3.1) and the sphere initialisation of the
// ablation (Sec. 4.3).
//
// The file is compiled without floating-point contraction: every float64
// operation is rounded on its own, in the order written.
//
// depth_points: every sampled pixel is back-projected (float64) and inserted by its voxel key into an open-addressing hash
// table in the workspace (64-bit key CAS, linear probing, table at least
// twice the number of pixels so every probe sequence ends); the slot keeps
// the lowest pixel index by atomic min.  A pixel is its voxel's
// representative when the slot holds its index; representatives are numbered
// in pixel order by a per-block count, a one-workgroup scan of the counts and
// a ballot rank inside each wave, and written compacted.
//
// plane_init_points: brute-force nearest neighbour of the K selected points
// (LDS tiles of 256 points, float64), radii and the rotation from the normal.
// plane_init_sphere: one-workgroup box and radius reduction, then one thread
// per plane.
#include "ps_internal.h"

using namespace ps;

namespace {

constexpr unsigned long long kEmpty = ~0ull;
constexpr long long kRange = 1ll << 20;
constexpr int kBlock = 256;

struct Sample {
  int n_cand;         // sampled pixels over all views
  int ws_, hs_;       // sampled columns and rows per view
  int H, W, stride;
  double voxel;
};

__device__ inline size_t map_index(int v, int c, int H, int W, int j, int i) {
  return (((size_t)v * 3 + c) * H + j) * W + i;
}

// Point, normal and voxel key of sampled pixel g; false when the pixel does
// not count.  Each operation is rounded on its own, in the order written.
__device__ bool back_project(const Sample& s, const float* __restrict__ depth, const float* __restrict__ normal,
                             const ps_camera* __restrict__ cams, int g, double p[3], double nw[3],
                             unsigned long long& key) {
  const int per_view = s.ws_ * s.hs_;
  const int v = g / per_view;
  const int r = g - v * per_view;
  const int j = (r / s.ws_) * s.stride;
  const int i = (r - (r / s.ws_) * s.ws_) * s.stride;
  const double d = (double)depth[((size_t)v * s.H + j) * s.W + i];
  const double nx = (double)normal[map_index(v, 0, s.H, s.W, j, i)];
  const double ny = (double)normal[map_index(v, 1, s.H, s.W, j, i)];
  const double nz = (double)normal[map_index(v, 2, s.H, s.W, j, i)];
  const double nn = sqrt(nx * nx + ny * ny + nz * nz);
  if (!(d > 0.0 && nn >= 0.5)) return false;
  const ps_camera& cm = cams[v];
  const double z = d / nn;
  const double xc = ((double)i + 0.5 - (double)cm.cx) / (double)cm.fx;
  const double yc = ((double)j + 0.5 - (double)cm.cy) / (double)cm.fy;
  const double q0 = xc * z - (double)cm.t[0];
  const double q1 = yc * z - (double)cm.t[1];
  const double q2 = z - (double)cm.t[2];
  const double m0 = nx / nn, m1 = ny / nn, m2 = nz / nn;
  long long ix[3];
  bool inside = true;
  for (int c = 0; c < 3; ++c) {
    const double r0 = (double)cm.R[c], r1 = (double)cm.R[3 + c], r2 = (double)cm.R[6 + c];
    p[c] = r0 * q0 + r1 * q1 + r2 * q2;
    nw[c] = r0 * m0 + r1 * m1 + r2 * m2;
    const double f = floor(p[c] / s.voxel);
    inside = inside && fabs(f) < (double)kRange;
    ix[c] = inside ? (long long)f : 0;
  }
  if (!inside) return false;
  key = ((unsigned long long)(ix[0] + kRange) << 42) | ((unsigned long long)(ix[1] + kRange) << 21) |
        (unsigned long long)(ix[2] + kRange);
  return true;
}

__device__ inline unsigned hash_slot(unsigned long long key, unsigned mask) {
  return (unsigned)((key * 0x9E3779B97F4A7C15ull) >> 32) & mask;
}

__global__ void dp_clear_kernel(unsigned long long* keys, int* rep, unsigned n) {
  const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    keys[i] = kEmpty;
    rep[i] = INT_MAX;
  }
}

__global__ __launch_bounds__(kBlock) void dp_insert_kernel(Sample s, const float* depth, const float* normal,
                                                           const ps_camera* cams, unsigned long long* keys,
                                                           int* rep, unsigned mask, int* slot_of) {
  const int g = blockIdx.x * kBlock + threadIdx.x;
  if (g >= s.n_cand) return;
  double p[3], nw[3];
  unsigned long long key;
  if (!back_project(s, depth, normal, cams, g, p, nw, key)) {
    slot_of[g] = -1;
    return;
  }
  // at most n_cand keys in a table of more than 2 n_cand slots: an empty
  // slot is always reached
  unsigned h = hash_slot(key, mask);
  while (true) {
    const unsigned long long old = atomicCAS(&keys[h], kEmpty, key);
    if (old == kEmpty || old == key) break;
    h = (h + 1) & mask;
  }
  atomicMin(&rep[h], g);
  slot_of[g] = (int)h;
}

__device__ inline bool is_rep(const int* __restrict__ slot_of, const int* __restrict__ rep, int g, int n) {
  if (g >= n) return false;
  const int h = slot_of[g];
  return h >= 0 && rep[h] == g;
}

__global__ __launch_bounds__(kBlock) void dp_count_kernel(int n, const int* slot_of, const int* rep, int* counts) {
  const int g = blockIdx.x * kBlock + threadIdx.x;
  const int c = __syncthreads_count(is_rep(slot_of, rep, g, n));
  if (threadIdx.x == 0) counts[blockIdx.x] = c;
}

__global__ __launch_bounds__(1024) void dp_scan_kernel(const int* counts, int* first, int nb, int* n_out) {
  __shared__ int lds[40];
  int mx = 0;
  const long long total = block_scan(counts, first, nb, lds, mx);
  if (threadIdx.x == 0) *n_out = (int)total;
}

__global__ __launch_bounds__(kBlock) void dp_write_kernel(Sample s, const float* depth, const float* normal,
                                                          const ps_camera* cams, const int* slot_of, const int* rep,
                                                          const int* first, float* points, float* normals,
                                                          int cap) {
  __shared__ int wave_base[kBlock / 64];
  const int g = blockIdx.x * kBlock + threadIdx.x;
  const bool mine = is_rep(slot_of, rep, g, s.n_cand);
  const unsigned long long ballot = __ballot(mine);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) wave_base[wid] = __popcll(ballot);
  __syncthreads();
  if (!mine) return;
  int pos = first[blockIdx.x];
  for (int w = 0; w < wid; ++w) pos += wave_base[w];
  pos += __popcll(ballot & ((1ull << lane) - 1));
  if (pos >= cap) return;
  double p[3], nw[3];
  unsigned long long key;
  back_project(s, depth, normal, cams, g, p, nw, key);
  for (int c = 0; c < 3; ++c) {
    points[3 * (size_t)pos + c] = (float)p[c];
    normals[3 * (size_t)pos + c] = (float)nw[c];
  }
}

// Shortest rotation taking e_z to the direction of n, as (w, x, y, z).
__device__ void quat_from_normal(double nx, double ny, double nz, float q[4]) {
  const double ln = sqrt(nx * nx + ny * ny + nz * nz);
  nx = nx / ln; ny = ny / ln; nz = nz / ln;
  // 1 + n_z without cancellation for n_z < 0 (|n| = 1)
  double w = nz >= 0.0 ? 1.0 + nz : (nx * nx + ny * ny) / (1.0 - nz);
  double x = -ny, y = nx;
  if (w <= 0.0) { w = 0.0; x = 1.0; y = 0.0; }
  const double lq = sqrt(w * w + x * x + y * y);
  q[0] = (float)(w / lq);
  q[1] = (float)(x / lq);
  q[2] = (float)(y / lq);
  q[3] = 0.f;
}

__global__ __launch_bounds__(kBlock) void init_points_kernel(const float* points, const float* normals, int n,
                                                             const int32_t* sel, int K, float r_min, float* center,
                                                             float* quat, float* radii) {
  __shared__ double tile[3][kBlock];
  const int k = blockIdx.x * kBlock + threadIdx.x;
  const double qnan = __builtin_nan("");
  int sk = k < K ? sel[k] : -1;
  const bool ok = sk >= 0 && sk < n;
  double a[3] = {qnan, qnan, qnan};
  if (ok)
    for (int c = 0; c < 3; ++c) a[c] = (double)points[3 * (size_t)sk + c];
  double best = __builtin_inf();
  for (int base = 0; base < K; base += kBlock) {
    const int j = base + threadIdx.x;
    const int sj = j < K ? sel[j] : -1;
    const bool okj = sj >= 0 && sj < n;
    for (int c = 0; c < 3; ++c) tile[c][threadIdx.x] = okj ? (double)points[3 * (size_t)sj + c] : qnan;
    __syncthreads();
    const int m = min(kBlock, K - base);
    for (int t = 0; t < m; ++t) {
      const double dx = a[0] - tile[0][t], dy = a[1] - tile[1][t], dz = a[2] - tile[2][t];
      const double d2 = dx * dx + dy * dy + dz * dz;
      if (base + t != k && d2 < best) best = d2;
    }
    __syncthreads();
  }
  if (k >= K) return;
  if (!ok) {
    for (int c = 0; c < 3; ++c) center[3 * (size_t)k + c] = (float)qnan;
    for (int c = 0; c < 4; ++c) quat[4 * (size_t)k + c] = (float)qnan;
    for (int c = 0; c < 4; ++c) radii[4 * (size_t)k + c] = (float)qnan;
    return;
  }
  for (int c = 0; c < 3; ++c) center[3 * (size_t)k + c] = points[3 * (size_t)sk + c];
  const double half = 0.5 * sqrt(best);
  const float r = (float)(half > (double)r_min ? half : (double)r_min);
  for (int c = 0; c < 4; ++c) radii[4 * (size_t)k + c] = r;
  float q[4];
  quat_from_normal((double)normals[3 * (size_t)sk], (double)normals[3 * (size_t)sk + 1],
                   (double)normals[3 * (size_t)sk + 2], q);
  for (int c = 0; c < 4; ++c) quat[4 * (size_t)k + c] = q[c];
}

// ws: c[3], R (float64)
__global__ __launch_bounds__(1024) void sphere_fit_kernel(const float* points, int n, double* ws) {
  __shared__ float lo[3][16], hi[3][16];
  __shared__ double md[16];
  __shared__ double ctr[3];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  float l[3] = {__builtin_inff(), __builtin_inff(), __builtin_inff()};
  float h[3] = {-__builtin_inff(), -__builtin_inff(), -__builtin_inff()};
  for (int i = threadIdx.x; i < n; i += 1024)
    for (int c = 0; c < 3; ++c) {
      const float x = points[3 * (size_t)i + c];
      l[c] = fminf(l[c], x);
      h[c] = fmaxf(h[c], x);
    }
  for (int c = 0; c < 3; ++c) {
    for (int o = 32; o > 0; o >>= 1) {
      l[c] = fminf(l[c], __shfl_xor(l[c], o, 64));
      h[c] = fmaxf(h[c], __shfl_xor(h[c], o, 64));
    }
    if (lane == 0) { lo[c][wid] = l[c]; hi[c][wid] = h[c]; }
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int c = threadIdx.x;
    float a = lo[c][0], b = hi[c][0];
    for (int w = 1; w < 16; ++w) { a = fminf(a, lo[c][w]); b = fmaxf(b, hi[c][w]); }
    ctr[c] = 0.5 * ((double)a + (double)b);
  }
  __syncthreads();
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) {
    const double dx = (double)points[3 * (size_t)i] - ctr[0];
    const double dy = (double)points[3 * (size_t)i + 1] - ctr[1];
    const double dz = (double)points[3 * (size_t)i + 2] - ctr[2];
    const double d2 = dx * dx + dy * dy + dz * dz;
    m = d2 > m ? d2 : m;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double y = __shfl_xor(m, o, 64);
    m = y > m ? y : m;
  }
  if (lane == 0) md[wid] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = md[0];
    for (int w = 1; w < 16; ++w) b = md[w] > b ? md[w] : b;
    ws[0] = ctr[0]; ws[1] = ctr[1]; ws[2] = ctr[2];
    ws[3] = sqrt(b);
  }
}

__global__ __launch_bounds__(kBlock) void sphere_place_kernel(const double* ws, const float* dirs, int K, float radius,
                                                              float* center, float* quat, float* radii) {
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= K) return;
  double u[3];
  for (int c = 0; c < 3; ++c) u[c] = (double)dirs[3 * (size_t)k + c];
  const double lu = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  for (int c = 0; c < 3; ++c) u[c] = u[c] / lu;
  const double R = ws[3];
  for (int c = 0; c < 3; ++c) center[3 * (size_t)k + c] = (float)(ws[c] + R * u[c]);
  float q[4];
  quat_from_normal(-u[0], -u[1], -u[2], q);
  for (int c = 0; c < 4; ++c) quat[4 * (size_t)k + c] = q[c];
  for (int c = 0; c < 4; ++c) radii[4 * (size_t)k + c] = radius;
}

struct DpLayout {
  int n_cand, nb;
  unsigned table;     // power of two > 2 n_cand
  size_t off_keys, off_rep, off_slot, off_counts, off_first, bytes;
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool dp_layout(int V, int H, int W, int stride, DpLayout& L) {
  if (V < 1 || H < 1 || W < 1 || stride < 1) return false;
  const long long hs = (H + stride - 1) / stride, wsz = (W + stride - 1) / stride;
  const long long n = (long long)V * hs * wsz;
  if (n > (1ll << 29)) return false;
  L.n_cand = (int)n;
  L.nb = (int)((n + kBlock - 1) / kBlock);
  unsigned t = 1024;
  while ((long long)t <= 2 * n) t <<= 1;
  L.table = t;
  size_t o = 0;
  L.off_keys = o; o = align256(o + 8 * (size_t)t);
  L.off_rep = o; o = align256(o + 4 * (size_t)t);
  L.off_slot = o; o = align256(o + 4 * (size_t)n);
  L.off_counts = o; o = align256(o + 4 * (size_t)(L.nb + 1));
  L.off_first = o; o = align256(o + 4 * (size_t)(L.nb + 1));
  L.bytes = o;
  return true;
}

}  // namespace

extern "C" size_t depth_points_ws_bytes(int V, int H, int W, int stride) {
  DpLayout L;
  return dp_layout(V, H, W, stride, L) ? L.bytes : 0;
}

extern "C" int depth_points(const float* depth, const float* normal, const ps_camera* cams, int V, int H, int W,
                            int stride, float voxel, float* points, float* normals, int cap, int32_t* n_out,
                            void* ws, size_t ws_bytes, void* stream) {
  DpLayout L;
  if (!depth || !normal || !cams || !n_out || !ws || cap < 0 || (cap > 0 && (!points || !normals)) ||
      !(voxel > 0.f) || !dp_layout(V, H, W, stride, L))
    return ps_set_error(PS_ERR_INVALID, "depth_points: bad argument");
  if (ws_bytes < L.bytes)
    return ps_set_error(PS_ERR_INVALID, "depth_points: workspace of %zu bytes, %zu needed", ws_bytes, L.bytes);
  char* base = (char*)ws;
  auto* keys = (unsigned long long*)(base + L.off_keys);
  auto* rep = (int*)(base + L.off_rep);
  auto* slot_of = (int*)(base + L.off_slot);
  auto* counts = (int*)(base + L.off_counts);
  auto* first = (int*)(base + L.off_first);
  Sample s;
  s.n_cand = L.n_cand;
  s.hs_ = (H + stride - 1) / stride;
  s.ws_ = (W + stride - 1) / stride;
  s.H = H; s.W = W; s.stride = stride;
  s.voxel = (double)voxel;
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(dp_clear_kernel, dim3((L.table + 255) / 256), dim3(256), 0, st, keys, rep, L.table);
  hipLaunchKernelGGL(dp_insert_kernel, dim3(L.nb), dim3(kBlock), 0, st, s, depth, normal, cams, keys, rep,
                     L.table - 1, slot_of);
  hipLaunchKernelGGL(dp_count_kernel, dim3(L.nb), dim3(kBlock), 0, st, L.n_cand, slot_of, rep, counts);
  hipLaunchKernelGGL(dp_scan_kernel, dim3(1), dim3(1024), 0, st, counts, first, L.nb, n_out);
  hipLaunchKernelGGL(dp_write_kernel, dim3(L.nb), dim3(kBlock), 0, st, s, depth, normal, cams, slot_of, rep, first,
                     points, normals, cap);
  PS_HIP_CHECK(hipGetLastError());
  return PS_OK;
}

extern "C" int plane_init_points(const float* points, const float* normals, int n, const int32_t* sel, int K,
                                 float r_min, float* center, float* quat, float* radii, void* stream) {
  if (!points || !normals || !sel || !center || !quat || !radii || K < 2 || n < 1)
    return ps_set_error(PS_ERR_INVALID, "plane_init_points: bad argument");
  hipLaunchKernelGGL(init_points_kernel, dim3((K + kBlock - 1) / kBlock), dim3(kBlock), 0, (hipStream_t)stream,
                     points, normals, n, sel, K, r_min, center, quat, radii);
  PS_HIP_CHECK(hipGetLastError());
  return PS_OK;
}

extern "C" int plane_init_sphere(const float* points, int n, const float* dirs, int K, float radius, float* center,
                                 float* quat, float* radii, void* ws, void* stream) {
  if (!points || !dirs || !center || !quat || !radii || !ws || n < 1 || K < 1)
    return ps_set_error(PS_ERR_INVALID, "plane_init_sphere: bad argument");
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(sphere_fit_kernel, dim3(1), dim3(1024), 0, st, points, n, (double*)ws);
  hipLaunchKernelGGL(sphere_place_kernel, dim3((K + kBlock - 1) / kBlock), dim3(kBlock), 0, st, (const double*)ws,
                     dirs, K, radius, center, quat, radii);
  PS_HIP_CHECK(hipGetLastError());
  return PS_OK;
}
