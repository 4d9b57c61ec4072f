// plane_render_fwd_noalloc: plane_project -> tile_bin -> plane_render_fwd of
// one render job with its workspace in a static device array instead of a
// caller-allocated buffer, for callers that cannot allocate device memory.
//
// The array lives in the library's code object: every GPU the library runs
// on holds its own copy, at its own address, from module load until the
// process ends.  Host code never passes the array's name to a kernel (on the
// host it is only a stand-in for the symbol); the device address comes from
// hipGetSymbolAddress, taken once per device with that device current, and
// is what the kernels receive, exactly as they receive a caller's workspace.
#include <mutex>
#include <string.h>

#include "ps_internal.h"

using namespace ps;

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;   // PS_NOALLOC_SCRATCH_BYTES
static_assert(kScratchBytes == PS_NOALLOC_SCRATCH_BYTES, "header and source agree on the scratch size");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
void* g_ptr[kMaxDevices];
hipError_t g_err[kMaxDevices];
std::once_flag g_once[kMaxDevices];

// Device address of this device's copy of the array (once per device).
int scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices)
    return ps_set_error(PS_ERR_INVALID, "plane_render_fwd_noalloc: device %d out of range", dev);
  std::call_once(g_once[dev], [dev]() {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
    void* p = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur >= 0 && cur != dev) {
      const hipError_t e2 = hipSetDevice(cur);
      if (e == hipSuccess) e = e2;
    }
    g_err[dev] = e;
    g_ptr[dev] = (e == hipSuccess) ? p : nullptr;
  });
  if (g_err[dev] != hipSuccess || !g_ptr[dev])
    return ps_set_error(PS_ERR_HIP, "plane_render_fwd_noalloc: hipGetSymbolAddress on device %d: %s", dev,
                        hipGetErrorString(g_err[dev]));
  *out = g_ptr[dev];
  return PS_OK;
}

// The slot table and the counters of the workspace (what ps_workspace_init
// writes), from kernel arguments: no host-to-device copy.
__global__ void noalloc_init_kernel(ps_slot slot, ps_slot* slots, long long* counters, unsigned long long* queue,
                                    int32_t* scan, int n_scan) {
  const int t = threadIdx.x;
  if (t == 0) slots[0] = slot;
  if (t < 64) counters[t] = 0;
  for (int i = t; i < 2 * 8 * 16; i += blockDim.x) queue[i] = 0ull;   // persistent-launch work queues
  for (int i = t; i < n_scan; i += blockDim.x) scan[i] = 0;           // binning-scan histogram and counters
}

// After the render: the binning overflowed (more pairs than the scratch
// holds) -> zero maps and PS_ERR_CAPACITY in *status; else PS_OK.
__global__ void noalloc_status_kernel(const long long* counters, float* depth, float* normal, int64_t n,
                                      int32_t* status) {
  const bool over = counters[C_OVERFLOW] != 0;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (over && i < n) {
    depth[i] = 0.f;
    normal[i] = 0.f;
    normal[n + i] = 0.f;
    normal[2 * n + i] = 0.f;
  }
  if (status && i == 0) *status = over ? PS_ERR_CAPACITY : PS_OK;
}

}  // namespace

extern "C" int plane_render_fwd_noalloc(const float* center, const float* quat, const float* radii, int K,
                                        const ps_camera* cam, int width, int height, int tile_w, int tile_h,
                                        const float* lambda, const ps_params* prm, float* depth, float* normal,
                                        int32_t* status, void* stream) {
  const char* who = "plane_render_fwd_noalloc";
  if (!cam || !lambda || !prm || !depth || !normal || K < 0 || (K > 0 && (!center || !quat || !radii)))
    return ps_set_error(PS_ERR_INVALID, "%s: null pointer or K < 0", who);
  if (!(prm->tau > 0.f && prm->tau < 1.f) || !(prm->z_near > 0.f) || prm->M < 1 || prm->M > kMaxM ||
      prm->weight_mode < 0 || prm->weight_mode > 2)
    return ps_set_error(PS_ERR_INVALID, "%s: bad ps_params", who);
  hipStream_t st = (hipStream_t)stream;
  // layout of one job with the largest pair capacity the scratch holds
  ps_slot slot;
  memset(&slot, 0, sizeof(slot));
  slot.plane_begin = 0;
  slot.plane_end = K;
  slot.cam = 0;
  slot.width = width;
  slot.height = height;
  slot.tile_w = tile_w;
  slot.tile_h = tile_h;
  ps_layout L;
  int rc = ps_layout_init(&slot, 1, 1, &L);
  if (rc) return rc;
  if (L.ws_bytes > kScratchBytes)
    return ps_set_error(PS_ERR_INVALID, "%s: %d planes at %dx%d need %zu bytes before any pair; the static "
                        "scratch holds %zu", who, K, width, height, L.ws_bytes, kScratchBytes);
  const size_t per_pair = 8 + 4 + 8 + 4 + 64 * (size_t)L.max_sub + sizeof(Rec);
  int64_t cap = (int64_t)((kScratchBytes - L.ws_bytes) / per_pair) + 1;
  if (cap > (int64_t(1) << 31) - 1) cap = (int64_t(1) << 31) - 1;
  for (;;) {
    rc = ps_layout_init(&slot, 1, cap, &L);
    if (rc) return rc;
    if (L.ws_bytes <= kScratchBytes) break;
    cap -= 64;   // region rounding: step back until the layout fits
    if (cap < 1) return ps_set_error(PS_ERR_INVALID, "%s: no pair fits in the static scratch", who);
  }
  int dev = 0;
  if (st) {
    hipDevice_t d;
    PS_HIP_CHECK(hipStreamGetDevice(st, &d));
    dev = (int)d;
  } else {
    PS_HIP_CHECK(hipGetDevice(&dev));
  }
  void* ws = nullptr;
  rc = scratch_address(dev, &ws);
  if (rc) return rc;
  char* base = (char*)ws;
  const int n_scan = (int)scan_words(L.n_tiles, L.n_records);
  hipLaunchKernelGGL(noalloc_init_kernel, dim3(1), dim3(256), 0, st, slot, (ps_slot*)(base + L.region[R_SLOTS]),
                     (long long*)(base + L.region[R_COUNTERS]), (unsigned long long*)(base + L.region[R_QUEUE]),
                     (int32_t*)(base + L.region[R_SCAN]), n_scan);
  PS_HIP_CHECK(hipGetLastError());
  rc = plane_project(&L, ws, center, quat, radii, K, cam, 1, lambda, prm, stream);
  if (rc) return rc;
  rc = tile_bin(&L, ws, nullptr, stream);
  if (rc) return rc;
  rc = plane_render_fwd(&L, ws, cam, 1, lambda, prm, depth, normal, nullptr, nullptr, stream);
  if (rc) return rc;
  const int64_t n = L.n_pixels;
  hipLaunchKernelGGL(noalloc_status_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                     (const long long*)(base + L.region[R_COUNTERS]), depth, normal, n, status);
  PS_HIP_CHECK(hipGetLastError());
  return PS_OK;
}
