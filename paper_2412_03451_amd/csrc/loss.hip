// loss_depth_normal: render loss of Eq. 14 and its gradient, per pixel.
//   l = a_cos |1 - N.N^| + a_nl1 sum_c |N_c - N^_c| + a_d |D - D^|
//   dl/dD = a_d sgn(D - D^)
//   dl/dN = -a_cos sgn(1 - N.N^) N^ + a_nl1 sgn(N - N^)      (sgn(0) = 0)
// The dot product is formed in float64 (products of float32 values are exact
// there), so the sign decision of the first term matches a float64 reference.
// One wave per 8x8 block writes its four partial sums (three terms and the
// plain |D - D^| sum) in float64; a second pass sums the blocks of each job in
// a fixed order.  Memory-bound: 32 bytes read and 16 written per pixel.
#include "ps_internal.h"

using namespace ps;

int ps_check_ws(const ps_layout* L, const void* ws, const char* who);

namespace {

struct LossArgs {
  const ps_slot* slots;
  int S, n_items;
  const float* D;
  const float* N;
  const float* Dt;
  const float* Nt;
  const uint8_t* mask;
  const int64_t* tgt_off;   // null: targets laid out like the jobs; else per-camera pixel offsets
  int n_cams;
  float a_cos, a_nl1, a_d;
  float* gD;
  float* gN;
  double* part;
  float* loss;
};

__device__ inline float sgnf(float x) { return x > 0.f ? 1.f : (x < 0.f ? -1.f : 0.f); }
__device__ inline double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// grid (items of the largest job / 4, jobs): the job is blockIdx.y, no search
__global__ __launch_bounds__(256) void loss_kernel(LossArgs a) {
  const int s = blockIdx.y;
  const ps_slot sl = a.slots[s];
  const int local = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int n_local = (s + 1 < a.S ? a.slots[s + 1].item_begin : a.n_items) - sl.item_begin;
  if (local >= n_local) return;
  const int item = sl.item_begin + local;
  const int sub_w = sl.tile_w >> 3;
  const int sub_per = sub_w * (sl.tile_h >> 3);
  const int tile = local / sub_per, sub = local - tile * sub_per;
  const int px = (tile % sl.tiles_x) * sl.tile_w + (sub % sub_w) * 8 + (lane & 7);
  const int py = (tile / sl.tiles_x) * sl.tile_h + (sub / sub_w) * 8 + (lane >> 3);
  double l0 = 0, l1 = 0, l2 = 0, l3 = 0;
  // targets of a camera: its own image at tgt_off[cam] (a camera whose
  // index is out of range contributes nothing)
  const bool valid = !a.tgt_off || (sl.cam >= 0 && sl.cam < a.n_cams);
  if (px < sl.width && py < sl.height && valid) {
    const int64_t HW = (int64_t)sl.width * sl.height;
    const int64_t local = (int64_t)py * sl.width + px;
    const int64_t p = sl.pix_off + local;
    const int64_t nb = 3 * sl.pix_off + local;
    const int64_t tp = a.tgt_off ? a.tgt_off[sl.cam] + local : p;
    const int64_t tnb = a.tgt_off ? 3 * a.tgt_off[sl.cam] + local : nb;
    const float m = a.mask ? (a.mask[tp] ? 1.f : 0.f) : 1.f;
    const float D = a.D[p], Dt = a.Dt[tp];
    float N[3], Nt[3];
    for (int c = 0; c < 3; ++c) {
      N[c] = a.N[nb + c * HW];
      Nt[c] = a.Nt[tnb + c * HW];
    }
    const double dot = (double)N[0] * Nt[0] + (double)N[1] * Nt[1] + (double)N[2] * Nt[2];
    const double e1 = 1.0 - dot;
    const float s1 = e1 > 0 ? 1.f : (e1 < 0 ? -1.f : 0.f);
    const float ed = D - Dt;
    a.gD[p] = m * a.a_d * sgnf(ed);
    double nl1 = 0;
    for (int c = 0; c < 3; ++c) {
      const float ec = N[c] - Nt[c];
      nl1 += fabs((double)N[c] - (double)Nt[c]);
      a.gN[nb + c * HW] = m * (-a.a_cos * s1 * Nt[c] + a.a_nl1 * sgnf(ec));
    }
    if (m != 0.f) {
      l0 = a.a_cos * fabs(e1);
      l1 = a.a_nl1 * nl1;
      l3 = fabs((double)D - (double)Dt);
      l2 = a.a_d * l3;
    }
  } else if (px < sl.width && py < sl.height) {
    const int64_t HW = (int64_t)sl.width * sl.height;
    const int64_t p = sl.pix_off + (int64_t)py * sl.width + px;
    const int64_t nb = 3 * sl.pix_off + (p - sl.pix_off);
    a.gD[p] = 0.f;
    for (int c = 0; c < 3; ++c) a.gN[nb + c * HW] = 0.f;
  }
  l0 = wave_sum_d(l0); l1 = wave_sum_d(l1); l2 = wave_sum_d(l2); l3 = wave_sum_d(l3);
  if (lane == 0) {
    double* o = a.part + 4 * (size_t)item;
    o[0] = l0; o[1] = l1; o[2] = l2; o[3] = l3;
  }
}

// One 256-thread workgroup per job: strided partial sums, wave sums, then the
// four wave results added in a fixed order (deterministic).
__global__ __launch_bounds__(256) void loss_reduce_kernel(LossArgs a) {
  __shared__ double lds[4][4];
  const int s = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int i0 = a.slots[s].item_begin;
  const int i1 = (s + 1 < a.S) ? a.slots[s + 1].item_begin : a.n_items;
  double acc[4] = {0, 0, 0, 0};
  for (int i = i0 + tid; i < i1; i += 256) {
    const double4 p = *reinterpret_cast<const double4*>(a.part + 4 * (size_t)i);
    acc[0] += p.x; acc[1] += p.y; acc[2] += p.z; acc[3] += p.w;
  }
  for (int q = 0; q < 4; ++q) acc[q] = wave_sum_d(acc[q]);
  if (lane == 0)
    for (int q = 0; q < 4; ++q) lds[wid][q] = acc[q];
  __syncthreads();
  if (tid == 0)
    for (int q = 0; q < 4; ++q) a.loss[4 * s + q] = (float)(((lds[0][q] + lds[1][q]) + lds[2][q]) + lds[3][q]);
}

}  // namespace

static int loss_launch(const ps_layout* L, void* ws, const float* depth, const float* normal,
                       const float* tgt_depth, const float* tgt_normal, const uint8_t* mask,
                       const int64_t* tgt_off, int n_cams, float a_cos, float a_nl1,
                       float a_d, float* loss, float* g_depth, float* g_normal, void* stream, const char* who) {
  int rc = ps_check_ws(L, ws, who);
  if (rc) return rc;
  if (!depth || !normal || !tgt_depth || !tgt_normal || !loss || !g_depth || !g_normal)
    return ps_set_error(PS_ERR_INVALID, "%s: null pointer", who);
  char* base = (char*)ws;
  LossArgs a;
  a.slots = (const ps_slot*)(base + L->region[R_SLOTS]);
  a.S = L->n_slots;
  a.n_items = L->n_items;
  a.D = depth; a.N = normal; a.Dt = tgt_depth; a.Nt = tgt_normal; a.mask = mask;
  a.tgt_off = tgt_off; a.n_cams = n_cams;
  a.a_cos = a_cos; a.a_nl1 = a_nl1; a.a_d = a_d;
  a.gD = g_depth; a.gN = g_normal;
  a.part = (double*)(base + L->region[R_LOSS]);
  a.loss = loss;
  hipStream_t st = (hipStream_t)stream;
  if (a.n_items > 0)
    hipLaunchKernelGGL(loss_kernel, dim3((L->max_items + 3) / 4, a.S), dim3(256), 0, st, a);
  hipLaunchKernelGGL(loss_reduce_kernel, dim3(a.S), dim3(256), 0, st, a);
  PS_HIP_CHECK(hipGetLastError());
  return PS_OK;
}

extern "C" int loss_depth_normal(const ps_layout* L, void* ws, const float* depth, const float* normal,
                                 const float* tgt_depth, const float* tgt_normal, const uint8_t* mask,
                                 float a_cos, float a_nl1, float a_d, float* loss, float* g_depth,
                                 float* g_normal, void* stream) {
  return loss_launch(L, ws, depth, normal, tgt_depth, tgt_normal, mask, nullptr, 0, a_cos, a_nl1, a_d,
                     loss, g_depth, g_normal, stream, "loss_depth_normal");
}

extern "C" int loss_depth_normal_cam(const ps_layout* L, void* ws, const float* depth, const float* normal,
                                     const float* tgt_depth, const float* tgt_normal, const uint8_t* mask,
                                     const int64_t* tgt_off, int n_cams, float a_cos, float a_nl1, float a_d,
                                     float* loss, float* g_depth, float* g_normal, void* stream) {
  if (!tgt_off || n_cams <= 0)
    return ps_set_error(PS_ERR_INVALID, "loss_depth_normal_cam: null tgt_off or n_cams <= 0");
  return loss_launch(L, ws, depth, normal, tgt_depth, tgt_normal, mask, tgt_off, n_cams, a_cos, a_nl1,
                     a_d, loss, g_depth, g_normal, stream, "loss_depth_normal_cam");
}
