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
  LossView v;
  double* part;
  float* loss;
};

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
  double l[4] = {0, 0, 0, 0};
  if (px < sl.width && py < sl.height) {
    const int64_t HW = (int64_t)sl.width * sl.height;
    const int64_t loc = (int64_t)py * sl.width + px;
    const float D = a.D[sl.pix_off + loc];
    float N[3];
    for (int c = 0; c < 3; ++c) N[c] = a.N[3 * sl.pix_off + loc + c * HW];
    loss_pixel(a.v, sl, px, py, D, N, l);
  }
  for (int q = 0; q < 4; ++q) l[q] = wave_sum_double(l[q]);
  if (lane == 0) {
    double* o = a.part + 4 * (size_t)item;
    o[0] = l[0]; o[1] = l[1]; o[2] = l[2]; o[3] = l[3];
  }
}

// One 1024-thread workgroup per job: strided partial sums, wave sums, then
// the 16 wave results added in a fixed order (deterministic).
__global__ __launch_bounds__(1024) void loss_reduce_kernel(const ps_slot* slots, int S, int n_items,
                                                           const double* part, float* loss) {
  __shared__ double lds[16][4];
  const int s = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int i0 = slots[s].item_begin;
  const int i1 = (s + 1 < S) ? slots[s + 1].item_begin : n_items;
  double acc[4] = {0, 0, 0, 0};
  for (int i = i0 + tid; i < i1; i += 1024) {
    const double4 p = *reinterpret_cast<const double4*>(part + 4 * (size_t)i);
    acc[0] += p.x; acc[1] += p.y; acc[2] += p.z; acc[3] += p.w;
  }
  for (int q = 0; q < 4; ++q) acc[q] = wave_sum_double(acc[q]);
  if (lane == 0)
    for (int q = 0; q < 4; ++q) lds[wid][q] = acc[q];
  __syncthreads();
  if (tid < 4) {
    double t = lds[0][tid];
    for (int w = 1; w < 16; ++w) t += lds[w][tid];
    loss[4 * s + tid] = (float)t;
  }
}

}  // namespace

// Loss sums per job from the per-8x8-block partials of the loss workspace
// region (used by the loss calls and by the forward that forms the loss).
int ps_loss_reduce(const ps_layout* L, void* ws, float* loss, void* stream) {
  char* base = (char*)ws;
  hipLaunchKernelGGL(loss_reduce_kernel, dim3(L->n_slots), dim3(1024), 0, (hipStream_t)stream,
                     (const ps_slot*)(base + L->region[R_SLOTS]), L->n_slots, L->n_items,
                     (const double*)(base + L->region[R_LOSS]), loss);
  PS_HIP_CHECK(hipGetLastError());
  return PS_OK;
}

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
  a.D = depth; a.N = normal;
  a.v.Dt = tgt_depth; a.v.Nt = tgt_normal; a.v.mask = mask;
  a.v.tgt_off = tgt_off; a.v.n_cams = n_cams;
  a.v.a_cos = a_cos; a.v.a_nl1 = a_nl1; a.v.a_d = a_d;
  a.v.gD = g_depth; a.v.gN = g_normal;
  a.part = (double*)(base + L->region[R_LOSS]);
  a.loss = loss;
  hipStream_t st = (hipStream_t)stream;
  if (a.n_items > 0)
    hipLaunchKernelGGL(loss_kernel, dim3((L->max_items + 3) / 4, a.S), dim3(256), 0, st, a);
  PS_HIP_CHECK(hipGetLastError());
  return ps_loss_reduce(L, ws, loss, stream);
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
