// plane_merge: plane instances after the fit (Sec. 3.3).  The file is
// compiled without floating-point contraction: the pair test turns float64
// arithmetic into a boolean and rounds every operation on its own, in the
// order written.
//
// Rounds of hooking: every related pair whose planes sit in different trees
// links the larger root under the smaller one (atomic minimum on the parent
// pointer), then every pointer is compressed to its root.  A round that
// links nothing ends the loop; each productive round removes at least one
// root, and every root is the smallest index of its tree, so the final roots
// label the connected components by their smallest plane index.
#include "ps_internal.h"

using namespace ps;

namespace {

constexpr int kBlock = 256;

struct MergeArgs {
  const float* center;
  const float* quat;
  const float* scene_center;
  int K;
  double cos_thr, off_thr;
  double* n;     // [3][K]
  double* o;     // [K]
  int* parent;   // [K]
  int* flag;     // [2]: linked in this round, instance count
};

__global__ __launch_bounds__(kBlock) void merge_prep_kernel(MergeArgs a) {
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k == 0) a.flag[1] = 0;
  if (k >= a.K) return;
  double w = a.quat[4 * (size_t)k], x = a.quat[4 * (size_t)k + 1];
  double y = a.quat[4 * (size_t)k + 2], z = a.quat[4 * (size_t)k + 3];
  const double qn = sqrt(w * w + x * x + y * y + z * z);
  w = w / qn; x = x / qn; y = y / qn; z = z / qn;
  const double n0 = 2.0 * (x * z + w * y);
  const double n1 = 2.0 * (y * z - w * x);
  const double n2 = 1.0 - 2.0 * (x * x + y * y);
  const double p0 = a.center[3 * (size_t)k], p1 = a.center[3 * (size_t)k + 1], p2 = a.center[3 * (size_t)k + 2];
  const double c0 = a.scene_center[0], c1 = a.scene_center[1], c2 = a.scene_center[2];
  a.n[k] = n0;
  a.n[a.K + k] = n1;
  a.n[2 * (size_t)a.K + k] = n2;
  a.o[k] = (p0 - c0) * n0 + (p1 - c1) * n1 + (p2 - c2) * n2;
  a.parent[k] = k;
}

__device__ inline int find_root(const int* parent, int k) {
  int r = parent[k];
  while (true) {
    const int p = parent[r];
    if (p == r) return r;
    r = p;
  }
}

__global__ void merge_clear_kernel(int* flag) { flag[0] = 0; }

// One thread per plane i, the planes j > i in LDS tiles.
__global__ __launch_bounds__(kBlock) void merge_hook_kernel(MergeArgs a) {
  __shared__ double tn[3][kBlock];
  __shared__ double to[kBlock];
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const bool act = i < a.K;
  double ni[3] = {0.0, 0.0, 0.0}, oi = 0.0;
  if (act) {
    for (int c = 0; c < 3; ++c) ni[c] = a.n[(size_t)c * a.K + i];
    oi = a.o[i];
  }
  bool linked = false;
  for (int base = blockIdx.x * kBlock; base < a.K; base += kBlock) {
    const int j = base + threadIdx.x;
    if (j < a.K) {
      for (int c = 0; c < 3; ++c) tn[c][threadIdx.x] = a.n[(size_t)c * a.K + j];
      to[threadIdx.x] = a.o[j];
    }
    __syncthreads();
    const int m = min(kBlock, a.K - base);
    if (act) {
      for (int t = 0; t < m; ++t) {
        const int jj = base + t;
        if (jj <= i) continue;
        const double d = ni[0] * tn[0][t] + ni[1] * tn[1][t] + ni[2] * tn[2][t];
        const double oj = d >= 0.0 ? to[t] : -to[t];
        if (fabs(d) > a.cos_thr && fabs(oi - oj) < a.off_thr) {
          const int ri = find_root(a.parent, i), rj = find_root(a.parent, jj);
          if (ri != rj) {
            atomicMin(&a.parent[max(ri, rj)], min(ri, rj));
            linked = true;
          }
        }
      }
    }
    __syncthreads();
  }
  if (__syncthreads_or(linked) && threadIdx.x == 0) atomicOr(&a.flag[0], 1);
}

__global__ __launch_bounds__(kBlock) void merge_compress_kernel(MergeArgs a, int32_t* label, int final_round) {
  const int k = blockIdx.x * kBlock + threadIdx.x;
  bool root = false;
  if (k < a.K) {
    const int r = find_root(a.parent, k);
    a.parent[k] = r;
    if (final_round) {
      label[k] = r;
      root = r == k;
    }
  }
  const int c = __syncthreads_count(root);
  if (final_round && threadIdx.x == 0 && c) atomicAdd(&a.flag[1], c);
}

__global__ void merge_count_kernel(const int* flag, int32_t* n_out) { *n_out = flag[1]; }

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

extern "C" size_t plane_merge_ws_bytes(int K) {
  if (K < 1) return 0;
  return align256(24 * (size_t)K) + align256(8 * (size_t)K) + align256(4 * (size_t)K) + 256;
}

extern "C" int plane_merge(const float* center, const float* quat, int K, const float* scene_center, double cos_thr,
                           double off_thr, int32_t* label, int32_t* n_out, void* ws, size_t ws_bytes, void* stream) {
  if (!center || !quat || !scene_center || !label || !n_out || !ws || K < 1 || !(off_thr >= 0.0))
    return ps_set_error(PS_ERR_INVALID, "plane_merge: bad argument");
  if (ws_bytes < plane_merge_ws_bytes(K))
    return ps_set_error(PS_ERR_INVALID, "plane_merge: workspace of %zu bytes, %zu needed", ws_bytes,
                        plane_merge_ws_bytes(K));
  MergeArgs a;
  a.center = center; a.quat = quat; a.scene_center = scene_center; a.K = K;
  a.cos_thr = cos_thr; a.off_thr = off_thr;
  char* base = (char*)ws;
  a.n = (double*)base; base += align256(24 * (size_t)K);
  a.o = (double*)base; base += align256(8 * (size_t)K);
  a.parent = (int*)base; base += align256(4 * (size_t)K);
  a.flag = (int*)base;
  hipStream_t st = (hipStream_t)stream;
  const unsigned g = (unsigned)((K + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(merge_prep_kernel, dim3(g), dim3(kBlock), 0, st, a);
  // every productive round removes a root: at most K rounds
  for (int round = 0; round <= K; ++round) {
    hipLaunchKernelGGL(merge_clear_kernel, dim3(1), dim3(1), 0, st, a.flag);
    hipLaunchKernelGGL(merge_hook_kernel, dim3(g), dim3(kBlock), 0, st, a);
    hipLaunchKernelGGL(merge_compress_kernel, dim3(g), dim3(kBlock), 0, st, a, label, 0);
    int linked = 0;
    PS_HIP_CHECK(hipMemcpyAsync(&linked, a.flag, sizeof(int), hipMemcpyDeviceToHost, st));
    PS_HIP_CHECK(hipStreamSynchronize(st));
    if (!linked) break;
  }
  hipLaunchKernelGGL(merge_compress_kernel, dim3(g), dim3(kBlock), 0, st, a, label, 1);
  hipLaunchKernelGGL(merge_count_kernel, dim3(1), dim3(1), 0, st, a.flag, n_out);
  PS_HIP_CHECK(hipGetLastError());
  return PS_OK;
}
