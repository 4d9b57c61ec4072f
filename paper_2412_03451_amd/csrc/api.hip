// Host-side plumbing of the C ABI: error messages, batch layout, workspace.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "ps_internal.h"

static thread_local char g_err[512] = "";

extern "C" int ps_set_error(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

extern "C" const char* ps_last_error(void) { return g_err; }

static bool tile_ok(int tw, int th) {
  return (tw == 8 && th == 8) || (tw == 16 && th == 16) || (tw == 32 && th == 8);
}

extern "C" int ps_layout_init(ps_slot* slots, int n_slots, int64_t pair_capacity, ps_layout* out) {
  if (!slots || !out || n_slots <= 0)
    return ps_set_error(PS_ERR_INVALID, "ps_layout_init: null pointer or n_slots <= 0");
  if (n_slots > 32767)   // the render items keep the job index as int16
    return ps_set_error(PS_ERR_INVALID, "ps_layout_init: more than 32767 jobs");
  if (pair_capacity < 1 || pair_capacity > (int64_t(1) << 31) - 1)
    return ps_set_error(PS_ERR_INVALID, "ps_layout_init: pair_capacity %lld out of range",
                        (long long)pair_capacity);
  memset(out, 0, sizeof(*out));
  int64_t rec = 0, tiles = 0, items = 0, pix = 0;
  int max_sub = 1, n_planes = 0, max_items = 0, max_chunks = 1;
  for (int s = 0; s < n_slots; ++s) {
    ps_slot& sl = slots[s];
    if (sl.plane_begin < 0 || sl.plane_end < sl.plane_begin)
      return ps_set_error(PS_ERR_INVALID, "slot %d: bad plane range [%d, %d)", s, sl.plane_begin,
                          sl.plane_end);
    if (sl.width <= 0 || sl.height <= 0 || sl.width > 32767 || sl.height > 32767)
      return ps_set_error(PS_ERR_INVALID, "slot %d: bad image size %dx%d", s, sl.width, sl.height);
    if (!tile_ok(sl.tile_w, sl.tile_h))
      return ps_set_error(PS_ERR_INVALID, "slot %d: tile %dx%d not one of 8x8, 16x16, 32x8", s,
                          sl.tile_w, sl.tile_h);
    if (sl.cam < 0) return ps_set_error(PS_ERR_INVALID, "slot %d: negative camera index", s);
    sl.tiles_x = (sl.width + sl.tile_w - 1) / sl.tile_w;
    sl.tiles_y = (sl.height + sl.tile_h - 1) / sl.tile_h;
    const int sub = (sl.tile_w / 8) * (sl.tile_h / 8);
    if (sub > max_sub) max_sub = sub;
    sl.rec_begin = (int32_t)rec;
    sl.tile_begin = (int32_t)tiles;
    sl.item_begin = (int32_t)items;
    sl.pix_off = pix;
    sl.pad = 0;
    rec += sl.plane_end - sl.plane_begin;
    tiles += (int64_t)sl.tiles_x * sl.tiles_y;
    items += (int64_t)sl.tiles_x * sl.tiles_y * sub;
    if (sl.tiles_x * sl.tiles_y * sub > max_items) max_items = sl.tiles_x * sl.tiles_y * sub;
    if ((sl.tiles_x * sl.tiles_y + 63) / 64 > max_chunks) max_chunks = (sl.tiles_x * sl.tiles_y + 63) / 64;
    pix += (int64_t)sl.width * sl.height;
    if (sl.plane_end > n_planes) n_planes = sl.plane_end;
  }
  if (rec >= (int64_t(1) << 31) || tiles >= (int64_t(1) << 30) || items >= (int64_t(1) << 31))
    return ps_set_error(PS_ERR_INVALID, "ps_layout_init: batch too large");
  out->n_slots = n_slots;
  out->n_records = (int32_t)rec;
  out->n_tiles = (int32_t)tiles;
  out->n_items = (int32_t)items;
  out->n_pixels = pix;
  out->pair_capacity = pair_capacity;
  out->max_sub = max_sub;
  out->max_items = max_items;
  out->max_chunks = max_chunks;
  out->slots_sorted = 1;
  for (int s = 1; s < n_slots; ++s)
    if (slots[s].plane_begin < slots[s - 1].plane_begin || slots[s].plane_end < slots[s - 1].plane_end)
      out->slots_sorted = 0;
  out->n_planes = n_planes;
  const size_t R = (size_t)rec, T = (size_t)tiles, C = (size_t)pair_capacity;
  const size_t sizes[PS_NUM_REGIONS] = {
      sizeof(ps_slot) * n_slots,       // R_SLOTS
      sizeof(ps::Rec) * (R + 1),       // R_REC
      sizeof(ps::BinRec) * (R + 1),    // R_BINREC
      4 * (R + 1),                     // R_REC_CNT
      4 * (R + 1),                     // R_REC_OFF
      4 * (T + 1),                     // R_TILE_CNT
      4 * (T + 1),                     // R_TILE_OFF
      4 * (T + 1),                     // R_TILE_CUR
      8 * C,                           // R_KEYS_U
      4 * C,                           // R_EMIT_U
      8 * C,                           // R_KEYS_S
      4 * C,                           // R_EMIT_S
      8 * 64,                          // R_COUNTERS
      64 * C * (size_t)max_sub,        // R_PARTIAL
      32 * ((size_t)items + 1),        // R_LOSS
      4 * (T + 1),                     // R_BIGTILES
      sizeof(ps::ItemDesc) * ((size_t)items + 1),  // R_ITEMS
      sizeof(ps::Rec) * C,             // R_RECS_S
      8 * ps::D_NUM * ((size_t)items + 1),  // R_DIAG
      4 * (T + 1),                     // R_TILEPOS
      4 * (R * (size_t)max_chunks + 1),  // R_CHUNK_CNT
      8 * 2 * 8 * 16,                  // R_QUEUE
      4 * (size_t)ps::scan_words(T, R),  // R_SCAN
      4 * (T + 1),                     // R_TILESLOT
  };
  size_t off = 0;
  for (int i = 0; i < PS_NUM_REGIONS; ++i) {
    out->region[i] = off;
    off = ps::align256(off + sizes[i]);
  }
  out->ws_bytes = off;
  return PS_OK;
}

extern "C" size_t ps_workspace_bytes(const ps_layout* L) { return L ? L->ws_bytes : 0; }

__global__ void ps_fill_i32(int32_t* p, int64_t n, int32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void ps_set_cams_kernel(ps_slot* slots, int S, const int32_t* view) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < S) slots[s].cam = view[s];
}

int ps_check_ws(const ps_layout* L, const void* ws, const char* who) {
  if (!L || !ws) return ps_set_error(PS_ERR_INVALID, "%s: null layout or workspace", who);
  if (((uintptr_t)ws) & 255) return ps_set_error(PS_ERR_INVALID, "%s: workspace not 256-byte aligned", who);
  if (L->n_slots <= 0 || L->ws_bytes == 0) return ps_set_error(PS_ERR_INVALID, "%s: empty layout", who);
  return PS_OK;
}

extern "C" int ps_workspace_init(const ps_layout* L, const ps_slot* slots, void* ws, void* stream) {
  int rc = ps_check_ws(L, ws, "ps_workspace_init");
  if (rc) return rc;
  if (!slots) return ps_set_error(PS_ERR_INVALID, "ps_workspace_init: null slots");
  hipStream_t st = (hipStream_t)stream;
  char* base = (char*)ws;
  PS_HIP_CHECK(hipMemcpyAsync(base + L->region[ps::R_SLOTS], slots, sizeof(ps_slot) * L->n_slots,
                              hipMemcpyHostToDevice, st));
  const int64_t n = 2 * 64;  // counters as int32 words
  hipLaunchKernelGGL(ps_fill_i32, dim3((n + 255) / 256), dim3(256), 0, st,
                     (int32_t*)(base + L->region[ps::R_COUNTERS]), n, 0);
  const int64_t nq = 2 * 2 * 8 * 16;  // work-queue counters as int32 words
  hipLaunchKernelGGL(ps_fill_i32, dim3((nq + 255) / 256), dim3(256), 0, st,
                     (int32_t*)(base + L->region[ps::R_QUEUE]), nq, 0);
  const int64_t ns = ps::scan_words(L->n_tiles, L->n_records);
  hipLaunchKernelGGL(ps_fill_i32, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, st,
                     (int32_t*)(base + L->region[ps::R_SCAN]), ns, 0);
  const int64_t nd = 2 * (int64_t)ps::D_NUM * (L->n_items + 1);  // statistics as int32 words
  hipLaunchKernelGGL(ps_fill_i32, dim3((unsigned)((nd + 255) / 256)), dim3(256), 0, st,
                     (int32_t*)(base + L->region[ps::R_DIAG]), nd, 0);
  PS_HIP_CHECK(hipGetLastError());
  return PS_OK;
}

extern "C" int ps_set_cameras(const ps_layout* L, void* ws, const int32_t* view_of_slot, void* stream) {
  int rc = ps_check_ws(L, ws, "ps_set_cameras");
  if (rc) return rc;
  if (!view_of_slot) return ps_set_error(PS_ERR_INVALID, "ps_set_cameras: null view array");
  char* base = (char*)ws;
  hipLaunchKernelGGL(ps_set_cams_kernel, dim3((L->n_slots + 63) / 64), dim3(64), 0,
                     (hipStream_t)stream, (ps_slot*)(base + L->region[ps::R_SLOTS]), L->n_slots,
                     view_of_slot);
  PS_HIP_CHECK(hipGetLastError());
  return PS_OK;
}

// One fitting iteration's device-side bookkeeping (captured with the step).
__global__ void ps_sched_kernel(ps_slot* slots, int S, int32_t* ite, const int32_t* table, int n_rows,
                                float* lambda, int32_t* step) {
  const int it = *ite;
  const int row = it % n_rows;
  for (int s = threadIdx.x; s < S; s += blockDim.x) slots[s].cam = table[(size_t)row * S + s];
  if (threadIdx.x == 0) {
    // Eq. 10, iteration counted from 0
    lambda[0] = (float)fmin(20.0 * exp(-(1.0 - 0.001 * it)), 300.0);
    step[0] = it + 1;
  }
  __syncthreads();
  if (threadIdx.x == 0) *ite = it + 1;
}

extern "C" int ps_fit_schedule(const ps_layout* L, void* ws, int32_t* ite, const int32_t* table, int n_rows,
                               float* lambda, int32_t* step, void* stream) {
  int rc = ps_check_ws(L, ws, "ps_fit_schedule");
  if (rc) return rc;
  if (!ite || !table || !lambda || !step) return ps_set_error(PS_ERR_INVALID, "ps_fit_schedule: null pointer");
  if (n_rows <= 0) return ps_set_error(PS_ERR_INVALID, "ps_fit_schedule: n_rows <= 0");
  char* base = (char*)ws;
  hipLaunchKernelGGL(ps_sched_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream,
                     (ps_slot*)(base + L->region[ps::R_SLOTS]), L->n_slots, ite, table, n_rows, lambda, step);
  PS_HIP_CHECK(hipGetLastError());
  return PS_OK;
}

// Sums and maxima of the per-block statistics into the counters (one
// workgroup, fixed order).
__global__ __launch_bounds__(1024) void ps_diag_reduce_kernel(const long long* diag, int n_items, long long* counters) {
  __shared__ long long red[32][11];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  long long sum[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  long long mx_steps = 0, mx_fwd = 0, mx_bwd = 0;
  for (int i = tid; i < n_items; i += 1024) {
    const long long* d = diag + (size_t)i * ps::D_NUM;
    for (int k = 0; k < 11; ++k) sum[k] += d[k];
    mx_steps = max(mx_steps, d[ps::D_STEPS]);
    mx_fwd = max(mx_fwd, d[ps::D_FWD_TICKS]);
    mx_bwd = max(mx_bwd, d[ps::D_BWD_TICKS]);
  }
  for (int o = 32; o >= 1; o >>= 1) {
    for (int k = 0; k < 11; ++k) sum[k] += __shfl_xor(sum[k], o, 64);
    mx_steps = max(mx_steps, __shfl_xor(mx_steps, o, 64));
    mx_fwd = max(mx_fwd, __shfl_xor(mx_fwd, o, 64));
    mx_bwd = max(mx_bwd, __shfl_xor(mx_bwd, o, 64));
  }
  if (lane == 0) {
    for (int k = 0; k < 11; ++k) red[wid][k] = sum[k];
    red[16 + wid][0] = mx_steps; red[16 + wid][1] = mx_fwd; red[16 + wid][2] = mx_bwd;
  }
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < 16; ++w) {
      for (int k = 0; k < 11; ++k) red[0][k] += red[w][k];
      for (int k = 0; k < 3; ++k) red[16][k] = max(red[16][k], red[16 + w][k]);
    }
    counters[ps::C_EVALS] = red[0][ps::D_EVALS];
    counters[ps::C_COMMITS] = red[0][ps::D_COMMITS];
    counters[ps::C_ITERS] = red[0][ps::D_STEPS];
    counters[ps::C_MAXITER] = red[16][0];
    counters[ps::C_WTIME] = red[0][ps::D_FWD_TICKS];
    counters[ps::C_WTMAX] = red[16][1];
    for (int k = 0; k < 4; ++k) counters[ps::C_BT_SETUP + k] = red[0][ps::D_BWD_SETUP + k];
    counters[ps::C_BG_CAND] = red[0][ps::D_BWD_CAND];
    counters[ps::C_BG_GROUPS] = red[0][ps::D_BWD_GROUPS];
    counters[ps::C_BT_MAX] = red[16][2];
  }
}

extern "C" int ps_read_counters(const ps_layout* L, void* ws, int64_t out[PS_N_COUNTERS], void* stream) {
  int rc = ps_check_ws(L, ws, "ps_read_counters");
  if (rc) return rc;
  if (!out) return ps_set_error(PS_ERR_INVALID, "ps_read_counters: null output");
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(ps_diag_reduce_kernel, dim3(1), dim3(1024), 0, st,
                     (const long long*)((char*)ws + L->region[ps::R_DIAG]), L->n_items,
                     (long long*)((char*)ws + L->region[ps::R_COUNTERS]));
  PS_HIP_CHECK(hipGetLastError());
  int64_t tmp[PS_N_COUNTERS];
  PS_HIP_CHECK(hipMemcpyAsync(tmp, (char*)ws + L->region[ps::R_COUNTERS], sizeof(tmp),
                              hipMemcpyDeviceToHost, st));
  PS_HIP_CHECK(hipStreamSynchronize(st));
  for (int i = 0; i < PS_N_COUNTERS; ++i) out[i] = tmp[i];
  return PS_OK;
}
