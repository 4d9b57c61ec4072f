// Internal definitions shared by the HIP kernels of the plane splatting library.
// Device-side record layouts, workspace regions and wave64 helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "planesplat.h"

namespace ps {

// ---------------------------------------------------------------------------
// Projection record: one per (plane, job).
//
// With the camera-frame pixel ray d_c(u, v) = ((u - cx)/fx, (v - cy)/fy, 1)
// (pixel center (u, v) = (i + 1/2, j + 1/2)) and the quantities of Frame
// below, the ray parameter of Eq. 4 and the in-plane coordinates of Eq. 6 are
//   t   = h / den,        den = d_c . nc          (d_c has z = 1: z-depth)
//   P_X = AX / den,       AX  = d_c . (h vxc - pvx nc)
//   P_Y = AY / den,       AY  = d_c . (h vyc - pvy nc)
// and den, AX, AY are affine in (u, v).  Their coefficients are kept in
// float64: the fringe of a rectangle is a few millimetres wide at
// lambda = 300 (sigmoid slope 1500 / m) while the ray meets it metres away, so
// float32 positions would already move fringe weights by ~1e-4.
// 128 bytes: two 64-byte scalar loads per candidate in the render loops.
struct alignas(16) Rec {
  double D0, Du, Dv;          // den(u, v) = D0 + Du u + Dv v
  double X0, Xu, Xv;          // AX(u, v)
  double Y0, Yu, Yv;          // AY(u, v)
  double h;                   // (p - o) . n
  float rxp, rxm, ryp, rym;   // radii (Eq. 1)
  float nx, ny, nz;           // rendered normal: R n, facing the camera
  int32_t cull;               // 1: no pixel of the job can see this record
  int16_t px0, py0, px1, py1; // inclusive pixel box of the grown footprint
  float pvx, pvy;             // (p - o) . vx, (p - o) . vy (backward only)
};
static_assert(sizeof(Rec) == 128, "Rec must stay 128 bytes");

// The first 96 bytes of a Rec: everything the per-pixel evaluation reads.
struct RecHead {
  double D0, Du, Dv, X0, Xu, Xv, Y0, Yu, Yv, h;
  float rxp, rxm, ryp, rym;
};
static_assert(sizeof(RecHead) == 96 && offsetof(Rec, rxp) == offsetof(RecHead, rxp), "RecHead layout");

// LDS staging of one batch of kBatch candidates of a tile list (one wave,
// lanes 0 .. kBatch-1 fetch one each): head[k][slot] is the k-th 16-byte
// chunk of the slot's candidate record (the RecHead, then the rendered
// normal), so the lanes' stores are conflict-free and the walk reads one
// candidate with seven wave-uniform 16-byte reads.  (A 32-entry batch halves
// the buffer and lets ten backward workgroups share a compute unit instead
// of eight: the 64-room batch step gains 4 %, the room fit's deep first
// steps lose 3 %, its whole trajectory is unchanged.)
constexpr int kBatch = 64;
struct StageLds {
  float4 head[7][kBatch];
  float tlb[kBatch];
  int rec[kBatch];
  float2 pv[kBatch];     // (p - o) . vx, (p - o) . vy (backward only)
  uint32_t em[kBatch];   // emit index of the (record, tile) pair (backward only)
};
static_assert(offsetof(Rec, nx) == 96, "normal follows the head");

// Binning view of a record: the edges of the projected, near-clipped
// footprint polygon of the rectangle grown by the fringe margin, as signed
// distance lines (nx u + ny v + c >= 0 inside, |(nx, ny)| = 1, pixel units),
// and a depth lower bound.
struct alignas(16) BinRec {
  double edge[5][3];
  int32_t nedge;    // 0: culled; 3..5 edges; -1: degenerate polygon, box test only
  float tlb;        // min camera z over the clipped grown rectangle (rounded down)
  int32_t tx0, ty0, tx1, ty1;  // inclusive tile rectangle
  int32_t slot;
  int32_t pad[3];
};
static_assert(sizeof(BinRec) == 160, "BinRec size");

// Workspace regions (byte offsets in ps_layout.region).
enum Region {
  R_SLOTS = 0,   // ps_slot[S]
  R_REC,         // Rec[R]
  R_BINREC,      // BinRec[R]
  R_REC_CNT,     // int[R + 1]   tiles per record
  R_REC_OFF,     // int[R + 1]   exclusive scan of R_REC_CNT (emit index base) within scan chunks
                 //   (add the chunk's base from R_SCAN); [R] the total
  R_TILE_CNT,    // int[T + 1]   records per tile
  R_TILE_OFF,    // int[T + 1]   exclusive scan of R_TILE_CNT: within scan chunks until the tile
                 //   sort writes the full offset back; [T] the total
  R_TILE_CUR,    // int[T]       scatter cursors
  R_KEYS_U,      // uint64[C]    unsorted (depth bound, record) keys
  R_EMIT_U,      // uint32[C]    unsorted emit indices
  R_KEYS_S,      // uint64[C]    keys sorted per tile
  R_EMIT_S,      // uint32[C]    emit indices in sorted order
  R_COUNTERS,    // int64[64]
  R_PARTIAL,     // float[C][max_sub][16]  backward partials per (pair, 8x8 block)
  R_LOSS,        // double[n_items][4]     loss partials per 8x8 block
  R_BIGTILES,    // int[T]       tiles whose list exceeds the small sort
  R_ITEMS,       // ItemDesc[n_items]  per 8x8 block: list range, pixel origin, camera
  R_RECS_S,      // Rec[C]       record copies in tile-list order
  R_DIAG,        // int64[n_items][16]  per-block walk statistics (flags bit 6)
  R_TILEPOS,     // int[T]       first render item of each tile (longest lists first)
  R_CHUNK_CNT,   // int[R][max_chunks]  passing tiles per (record, group of 64 tiles of its box)
  R_QUEUE,       // uint64[2][8][16]  work-queue counters of persistent render launches (one line each)
  R_SCAN,        // int[2 G + (G + 1) kBuckets + 16]  binning scan: chunk bases of tile and record
                 //   offsets, per-chunk list-length histograms then each chunk's start in every
                 //   bucket, the totals per bucket, counters (zero between calls); G scan chunks
  R_TILESLOT,    // int[T + 1]   job slot of each tile (binning scan, for the tile sort)
  R_NUM_USED     // further regions are reserved (size 0)
};
// Render items are placed longest tile list first (buckets of list length),
// so the blocks that take longest start first.
constexpr int kBuckets = 1024;
// tiles and records per workgroup of the binning scan
constexpr int kScanChunk = 4096;
__host__ __device__ inline int scan_chunks(int64_t T, int64_t R) {
  const int64_t n = T > R ? T : R;
  return n > 0 ? (int)((n + kScanChunk - 1) / kScanChunk) : 1;
}
// int32 words of R_SCAN
__host__ __device__ inline int64_t scan_words(int64_t T, int64_t R) {
  const int64_t G = scan_chunks(T, R);
  return 2 * G + (G + 1) * kBuckets + 16;
}
__host__ __device__ inline int length_bucket(int n) { return n >> 2 < kBuckets - 1 ? n >> 2 : kBuckets - 1; }
// per-block statistics slots of R_DIAG
enum DiagSlot {
  D_EVALS = 0, D_COMMITS, D_STEPS, D_FWD_TICKS,
  D_BWD_SETUP, D_BWD_WALK, D_BWD_SORT, D_BWD_GRAD, D_BWD_CAND, D_BWD_GROUPS, D_BWD_TICKS,
  D_NUM = 16
};
static_assert(R_NUM_USED <= PS_NUM_REGIONS, "region table");

// Render item (one 8x8 pixel block), written by the binning sort so that a
// render block reaches its list with one load.
struct alignas(16) ItemDesc {
  int32_t b, e;              // range of the tile list in keys / record copies
  int16_t ox, oy;            // pixel origin of the block
  int16_t width, height;     // image size of the job
  int32_t cam;               // camera index of the job
  int16_t sub;               // 8x8 block index inside the tile
  int16_t slot;              // job of the block
  int64_t pix_off;           // first pixel of the job
};
static_assert(sizeof(ItemDesc) == 32, "ItemDesc size");

enum Counter {
  C_PAIRS = 0,     // pairs needed
  C_OVERFLOW = 1,  // nonzero: pairs exceed capacity or a tile exceeds the sort limit
  C_MAXTILE = 2,   // largest tile list
  C_SLOW = 3,      // pixels that took the exact fallback ordering path
  C_NBIG = 4,      // number of big tiles
  C_BWD_PASSES = 5, // extra backward recompute passes taken
  C_EVALS = 6,     // (pixel, candidate) pairs evaluated by the forward walk
  C_COMMITS = 7,   // hits composited by the forward walk
  C_ITERS = 8,     // candidate steps of the forward walk, summed over waves
  C_MAXITER = 9,   // candidate steps of the longest forward wave
  C_WTIME = 10,    // forward wave run time (100 MHz ticks), summed
  C_WTMAX = 11,    // longest forward wave run time
  C_BT_SETUP = 12, // backward phase times (ticks, summed over blocks)
  C_BT_WALK = 13,
  C_BT_SORT = 14,
  C_BT_GRAD = 15,
  C_BG_CAND = 16,  // candidates visited by the gradient pass
  C_BG_GROUPS = 17, // candidate groups fetched by the gradient pass
  C_STICKY = 18,   // nonzero once any tile_bin since ps_workspace_init overflowed
  C_BT_MAX = 19    // longest backward block run time (ticks)
};
static_assert(C_BT_MAX + 1 == PS_N_COUNTERS, "counter count");
constexpr int kFlagDiag = 64;   // params.flags bit 6: forward walk statistics
constexpr int kFlagNoPersist = 256;   // params.flags bit 8: one workgroup per item even for large batches
constexpr int kFlagPersistFwd = 512;  // params.flags bit 9: the forward persistent too
constexpr int kFlagReduceWave = 1024; // params.flags bit 10: the gradient reduction a wave per plane at any size
constexpr int kReduceWaveMin = 8192;  // planes from which the gradient reduction takes a wave per plane
constexpr int kFlagPathDiag = 128;   // params.flags bit 7: mark fallback-path pixels in the hit counts

constexpr int kMaxM = 30;
constexpr int kSmallSort = 256;   // tile lists up to this size sort in one wave (registers or 3 KB of LDS)
constexpr int kBigSort = 4096;    // tile lists up to this size sort in one LDS pass (48 KB of LDS);
                                  // longer ones sort in chunks of this size, then merge in memory
constexpr int kMaxList = 32767;   // longest tile list: list positions are kept as int16

inline __host__ __device__ size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// ---------------------------------------------------------------------------
// wave64 helpers
__device__ inline int lane_id() { return __lane_id(); }

// Cross-lane exchanges that stay on the VALU (no LDS round trip): DPP quad
// permutes (lane ^ 1, lane ^ 2) and row mirrors (lane ^ 7 inside 8 lanes,
// lane ^ 15 inside a 16-lane row), and the gfx950 permlane swaps, which
// exchange the odd 16-lane rows of one register with the even rows of
// another (lane ^ 16) or the upper half of one with the lower half of
// another (lane ^ 32).  The six partners reach every lane of the wave.
// Every lane must be active.
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppMirror16 = 0x140, kDppMirror8 = 0x141;
template <int CTRL>
__device__ inline int dpp_int(int v) {
  return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ inline float dpp_float(float v) {
  return __int_as_float(dpp_int<CTRL>(__float_as_int(v)));
}

// All-reduce over the wave; every lane receives the same bits (each step
// combines a lane with its partner by a commutative operation).
template <class T, class Op>
__device__ inline T wave_allreduce(T v, Op op) {
  static_assert(sizeof(T) == 4, "32-bit values");
  auto bits = [](T x) { return __builtin_bit_cast(unsigned, x); };
  auto back = [](unsigned x) { return __builtin_bit_cast(T, x); };
  v = op(v, back((unsigned)dpp_int<kDppXor1>((int)bits(v))));
  v = op(v, back((unsigned)dpp_int<kDppXor2>((int)bits(v))));
  v = op(v, back((unsigned)dpp_int<kDppMirror8>((int)bits(v))));
  v = op(v, back((unsigned)dpp_int<kDppMirror16>((int)bits(v))));
  const auto r16 = __builtin_amdgcn_permlane16_swap(bits(v), bits(v), false, false);
  v = op(back(r16[0]), back(r16[1]));
  const auto r32 = __builtin_amdgcn_permlane32_swap(bits(v), bits(v), false, false);
  return op(back(r32[0]), back(r32[1]));
}
__device__ inline float wave_sum(float v) {
  return wave_allreduce(v, [](float x, float y) { return x + y; });
}
__device__ inline int wave_min_int(int v) {
  return wave_allreduce(v, [](int x, int y) { return min(x, y); });
}
__device__ inline int wave_max_int(int v) {
  return wave_allreduce(v, [](int x, int y) { return max(x, y); });
}
__device__ inline uint64_t ballot(bool p) { return __ballot(p); }
__device__ inline int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Job lookup: largest s with slots[s].<field> <= x (slots sorted by field).
__device__ inline int find_slot_by_item(const ps_slot* __restrict__ sl, int S, int item) {
  int lo = 0, hi = S - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (sl[mid].item_begin <= item) lo = mid; else hi = mid - 1;
  }
  return lo;
}
__device__ inline int find_slot_by_tile(const ps_slot* __restrict__ sl, int S, int tile) {
  int lo = 0, hi = S - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (sl[mid].tile_begin <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}
__device__ inline int find_slot_by_rec(const ps_slot* __restrict__ sl, int S, int rec) {
  int lo = 0, hi = S - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (sl[mid].rec_begin <= rec) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Exclusive scan of in[0, n) into out[0, n], out[n] = total, by one
// 1024-thread workgroup: blocks of 4096 elements, 4 per thread, wave64
// inclusive scans by shuffles, wave totals through LDS, running carry.
__device__ inline long long block_scan(const int* __restrict__ in, int* __restrict__ out, int n, int* lds_wave,
                                int& maxv) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  long long carry = 0;
  int mx = 0;
  for (int base = 0; base < n; base += 4096) {
    int v[4];
    int local = 0;
    for (int j = 0; j < 4; ++j) {
      const int idx = base + tid * 4 + j;
      v[j] = idx < n ? in[idx] : 0;
      mx = max(mx, v[j]);
      local += v[j];
    }
    int incl = local;
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(incl, o, 64);
      if (lane >= o) incl += y;
    }
    if (lane == 63) lds_wave[wid] = incl;
    __syncthreads();
    if (wid == 0) {
      int x = lane < 16 ? lds_wave[lane] : 0;
      int xi = x;
      for (int o = 1; o < 16; o <<= 1) {
        const int y = __shfl_up(xi, o, 64);
        if (lane >= o) xi += y;
      }
      if (lane < 16) lds_wave[16 + lane] = xi - x;   // exclusive wave offsets
      if (lane == 15) lds_wave[32] = xi;             // block total
    }
    __syncthreads();
    int run = (int)carry + lds_wave[16 + wid] + (incl - local);
    for (int j = 0; j < 4; ++j) {
      const int idx = base + tid * 4 + j;
      if (idx < n) out[idx] = run;
      run += v[j];
    }
    carry += lds_wave[32];
    __syncthreads();
  }
  // max over the workgroup
  mx = wave_max_int(mx);
  if (lane == 0) lds_wave[wid] = mx;
  __syncthreads();
  if (tid == 0) {
    int m = 0;
    for (int w = 0; w < 16; ++w) m = max(m, lds_wave[w]);
    lds_wave[33] = m;
  }
  __syncthreads();
  maxv = lds_wave[33];
  if (tid == 0) out[n] = (int)carry;
  __syncthreads();
  return carry;
}

// float64 reciprocal: hardware estimate refined by two Newton steps.
__device__ inline double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
// One Newton step: the gfx950 estimate is within 5e-8 relative (measured
// over 2^20 values in [1e-3, 1e3]) and one step brings it to 2.2e-15, ample
// for the ray parameter and in-plane offsets (their float32 depth and float64
// fringe test need ~1e-9).
__device__ inline double rcp64_fast(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}

// Filter bound of the weight (closed form): modes 0 and 1, the fringe
// margin delta with w >= tau  <=>  a* >= -delta, delta = z / (5 lambda) with
// z = ln(2/tau - 1) (mode 0) or ln(1/tau - 1) (mode 1); mode 2 (the Gaussian
// of Eq. 5), Q with w >= tau  <=>  q <= Q, Q = 2 ln(1/tau).  The logarithm
// is a constant of the launch, taken on the host (filter_log); the kernels
// only divide by 5 lambda.
inline double filter_log(double tau, int mode) {
  if (mode == 2) return 2.0 * log(1.0 / tau);
  return (mode == 0) ? log(2.0 / tau - 1.0) : log(1.0 / tau - 1.0);
}
__device__ inline double fringe_margin(double lam, double flog, int mode) {
  return mode == 2 ? flog : flog / (5.0 * lam);
}

// Splat weight from a* (Eq. 7-9; mode 0 clamps the printed 2 sigmoid at 1)
// and omw = 1 - w formed from the same argument by an identity
// (1 - 2 s(z) = tanh(-z/2) = expm1(-z) / (expm1(-z) + 2), 1 - s(z) = s(-z)),
// not by a subtraction: behind a nearly opaque layer the transmittance keeps
// its relative precision.
__device__ inline float splat_weight(float a, float lam5, int mode, float& omw) {
  if (mode == 2) {   // Gaussian of Eq. 5, a = q: w = exp(-q/2), 1 - w = -expm1(-q/2)
    const float h = -0.5f * a;
    omw = -expm1f(h);
    return expf(h);
  }
  const float z = lam5 * a;
  if (mode == 0) {
    if (a >= 0.f) {
      omw = 0.f;
      return 1.f;
    }
    const float em = expm1f(-z);  // > 0
    const float r = __builtin_amdgcn_rcpf(em + 2.f);   // 1 ulp: both results keep their relative precision
    omw = em * r;
    return 2.f * r;
  }
  const float e = expf(-z);
  const float r = __builtin_amdgcn_rcpf(1.f + e);
  omw = e * r;
  return r;
}
// dw/da* (0 on the opaque side of mode 0).
__device__ inline float splat_weight_grad(float a, float w, float omw, float lam5, int mode) {
  if (mode == 0) return (a >= 0.f) ? 0.f : lam5 * w * (1.f - 0.5f * w);
  return lam5 * w * omw;
}

// Per-lane ray-plane evaluation in float64 (Eq. 4, 6, 7-9 up to a*).
struct PairGeom {
  double den, PX, PY, t;
  double a;        // a* = min(a_X, a_Y); mode 2: q = (P_X / r_X)^2 + (P_Y / r_Y)^2
  bool ok;         // valid hit in front of the near plane with w >= tau
  bool xbranch;    // a_X < a_Y: Eq. 9 takes w_X (tie -> w_Y)
};

template <bool GAUSS, class R>
__device__ inline PairGeom eval_pair(const R& r, double u, double v, double eps_den, double z_near,
                                     double delta) {
  PairGeom g;
  g.den = fma(r.Du, u, fma(r.Dv, v, r.D0));
  const double ax = fma(r.Xu, u, fma(r.Xv, v, r.X0));
  const double ay = fma(r.Yu, u, fma(r.Yv, v, r.Y0));
  const bool okd = fabs(g.den) > eps_den;
  const double rd = rcp64_fast(okd ? g.den : 1.0);
  g.t = r.h * rd;
  g.PX = ax * rd;
  g.PY = ay * rd;
  if (GAUSS) {   // weight mode 2, the Gaussian (Eq. 5): standard deviations the radii of the hit's side
    const double qx = g.PX / (g.PX > 0.0 ? (double)r.rxp : (double)r.rxm);
    const double qy = g.PY / (g.PY > 0.0 ? (double)r.ryp : (double)r.rym);
    g.a = qx * qx + qy * qy;
    g.xbranch = true;
    g.ok = okd && (g.t > z_near) && (g.a <= delta);
    return g;
  }
  const double aX = (g.PX > 0.0) ? (double)r.rxp - g.PX : (double)r.rxm + g.PX;
  const double aY = (g.PY > 0.0) ? (double)r.ryp - g.PY : (double)r.rym + g.PY;
  g.xbranch = aX < aY;
  g.a = g.xbranch ? aX : aY;
  g.ok = okd && (g.t > z_near) && (g.a >= -delta);
  return g;
}

// Render loss of Eq. 14 at one pixel and its gradient, shared by the loss
// kernel and the forward that forms the loss itself (same arithmetic, same
// bits):
//   l = a_cos |1 - N.N^| + a_nl1 sum_c |N_c - N^_c| + a_d |D - D^|,
//   dl/dD = a_d sgn(D - D^),  dl/dN = -a_cos sgn(1 - N.N^) N^ + a_nl1 sgn(N - N^)
// with sgn(0) = 0 and the dot product in float64 (products of float32 values
// are exact there).  Adds the pixel's three terms and |D - D^| to l[0..3].
struct LossView {
  const float* Dt;
  const float* Nt;
  const uint8_t* mask;
  const int64_t* tgt_off;   // null: targets laid out like the jobs; else per-camera pixel offsets
  int n_cams;
  float a_cos, a_nl1, a_d;
  float* gD;
  float* gN;
};

// One parameter's bias-corrected Adam update (Sec. 3.3), step t (1-based);
// m and v are updated in place, the new parameter is returned.  Shared by
// adam_step_planes and the reduction that applies Adam itself, so both give
// the same bits.  adam_bias forms the step's two bias corrections, which the
// reduction computes before its gradients are known.
__device__ inline void adam_bias(float b1, float b2, int t, double& bc1, double& bc2) {
  bc1 = 1.0 - pow((double)b1, (double)t);
  bc2 = 1.0 - pow((double)b2, (double)t);
}

__device__ inline float adam_apply(float p, float g, float& m, float& v, float lr, float b1, float b2, float eps,
                                   double bc1, double bc2) {
  m = b1 * m + (1.f - b1) * g;
  v = b2 * v + (1.f - b2) * g * g;
  const float mhat = (float)((double)m / bc1);
  const float vhat = (float)((double)v / bc2);
  return p - lr * mhat / (sqrtf(vhat) + eps);
}

__device__ inline float adam_update(float p, float g, float& m, float& v, float lr, float b1, float b2, float eps,
                                    int t) {
  double bc1, bc2;
  adam_bias(b1, b2, t, bc1, bc2);
  return adam_apply(p, g, m, v, lr, b1, b2, eps, bc1, bc2);
}

// float64 wave sum (the loss partials), in a fixed order
__device__ inline double wave_sum_double(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline float sgn_f(float x) { return x > 0.f ? 1.f : (x < 0.f ? -1.f : 0.f); }

// The targets of one pixel (read before the render needs them, so that their
// latency overlaps the walk).
struct LossTargets {
  float Dt, Nt[3], m;
  int64_t p, nb, HW;
  bool valid;
};

__device__ inline LossTargets loss_targets(const LossView& a, const ps_slot& sl, int px, int py) {
  LossTargets t;
  t.HW = (int64_t)sl.width * sl.height;
  const int64_t local = (int64_t)py * sl.width + px;
  t.p = sl.pix_off + local;
  t.nb = 3 * sl.pix_off + local;
  // targets of a camera: its own image at tgt_off[cam] (a camera whose
  // index is out of range contributes nothing)
  t.valid = !a.tgt_off || (sl.cam >= 0 && sl.cam < a.n_cams);
  t.Dt = 0.f;
  t.Nt[0] = t.Nt[1] = t.Nt[2] = 0.f;
  t.m = 0.f;
  if (!t.valid) return t;
  const int64_t tp = a.tgt_off ? a.tgt_off[sl.cam] + local : t.p;
  const int64_t tnb = a.tgt_off ? 3 * a.tgt_off[sl.cam] + local : t.nb;
  t.m = a.mask ? (a.mask[tp] ? 1.f : 0.f) : 1.f;
  t.Dt = a.Dt[tp];
  for (int c = 0; c < 3; ++c) t.Nt[c] = a.Nt[tnb + c * t.HW];
  return t;
}

// g (optional): the pixel's gradient as written, dl/dD then dl/dN.
__device__ inline void loss_apply(const LossView& a, const LossTargets& t, float D, const float N[3], double l[4],
                                  float* g = nullptr) {
  if (!t.valid) {
    if (a.gD) {
      a.gD[t.p] = 0.f;
      for (int c = 0; c < 3; ++c) a.gN[t.nb + c * t.HW] = 0.f;
    }
    if (g) g[0] = g[1] = g[2] = g[3] = 0.f;
    return;
  }
  const float m = t.m;
  const float* Nt = t.Nt;
  const double dot = (double)N[0] * Nt[0] + (double)N[1] * Nt[1] + (double)N[2] * Nt[2];
  const double e1 = 1.0 - dot;
  const float s1 = e1 > 0 ? 1.f : (e1 < 0 ? -1.f : 0.f);
  const float ed = D - t.Dt;
  const float gd = m * a.a_d * sgn_f(ed);
  if (a.gD) a.gD[t.p] = gd;   // (null: the caller keeps the gradient in registers only)
  if (g) g[0] = gd;
  double nl1 = 0;
  for (int c = 0; c < 3; ++c) {
    const float ec = N[c] - Nt[c];
    nl1 += fabs((double)N[c] - (double)Nt[c]);
    const float gn = m * (-a.a_cos * s1 * Nt[c] + a.a_nl1 * sgn_f(ec));
    if (a.gN) a.gN[t.nb + c * t.HW] = gn;
    if (g) g[1 + c] = gn;
  }
  if (m != 0.f) {
    const double ad = fabs((double)D - (double)t.Dt);
    l[0] += a.a_cos * fabs(e1);
    l[1] += a.a_nl1 * nl1;
    l[2] += a.a_d * ad;
    l[3] += ad;
  }
}

__device__ inline void loss_pixel(const LossView& a, const ps_slot& sl, int px, int py, float D, const float N[3],
                                  double l[4]) {
  loss_apply(a, loss_targets(a, sl, px, py), D, N, l);
}

__device__ inline int find_slot_by_pix(const ps_slot* __restrict__ sl, int S, int64_t pix_off) {
  int lo = 0, hi = S - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sl[mid].pix_off <= pix_off) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <class R>
__device__ inline PairGeom eval_pair_mode(const R& r, double u, double v, double eps_den, double z_near,
                                          double delta, int mode) {
  return mode == 2 ? eval_pair<true>(r, u, v, eps_den, z_near, delta)
                   : eval_pair<false>(r, u, v, eps_den, z_near, delta);
}

// Strict order of hits: float32 depth, then record index (= plane order).
__device__ inline bool key_less(float ta, int ia, float tb, int ib) {
  return ta < tb || (ta == tb && ia < ib);
}

}  // namespace ps

// error plumbing (api.hip)
extern "C" int ps_set_error(int code, const char* fmt, ...);
// Loss sums per job from the per-8x8-block partials of the loss region.
int ps_loss_reduce(const ps_layout* L, void* ws, float* loss, void* stream);
#define PS_HIP_CHECK(expr)                                                      \
  do {                                                                          \
    hipError_t _e = (expr);                                                     \
    if (_e != hipSuccess)                                                       \
      return ps_set_error(PS_ERR_HIP, "%s: %s", #expr, hipGetErrorString(_e));  \
  } while (0)

namespace ps {

// Frame of plane k as seen by one camera, float64.  The camera maps world to
// camera coordinates by x_c = R x + t; the ray of camera direction d_c starts
// at o = -R^T t with world direction d = R^T d_c (the matrix is float32 input,
// not exactly orthogonal, so everything is written with these exact
// identities and never with R^T R = I):
//   d . n   = d_c . (R n)                    -> nc = R n
//   (p - o) . n = p . n + t . (R n)          -> h
//   (p - o) . vx = p . vx + t . (R vx)       -> pvx (likewise pvy)
// so t = h / (d_c . nc) and P_X = (h (d_c . vxc) - pvx (d_c . nc)) / (d_c . nc).
struct Frame {
  double p[3], n[3], vx[3], vy[3];  // world center and local frame (Eq. 2-3)
  double nc[3], vxc[3], vyc[3];     // R n, R vx, R vy
  double h, pvx, pvy;
  double q[4];                      // normalised quaternion (w, x, y, z)
  double qnorm;                     // |q| before normalisation
};

__device__ inline bool plane_frame(const float* __restrict__ center, const float* __restrict__ quat,
                                   int k, const ps_camera& cam, Frame& f) {
  double w = quat[4 * k + 0], x = quat[4 * k + 1], y = quat[4 * k + 2], z = quat[4 * k + 3];
  const double qn = sqrt(w * w + x * x + y * y + z * z);
  f.qnorm = qn;
  if (!(qn > 1e-30)) return false;
  w /= qn; x /= qn; y /= qn; z /= qn;
  f.q[0] = w; f.q[1] = x; f.q[2] = y; f.q[3] = z;
  // columns of R(q)
  f.vx[0] = 1 - 2 * (y * y + z * z); f.vx[1] = 2 * (x * y + w * z); f.vx[2] = 2 * (x * z - w * y);
  f.vy[0] = 2 * (x * y - w * z); f.vy[1] = 1 - 2 * (x * x + z * z); f.vy[2] = 2 * (y * z + w * x);
  f.n[0] = 2 * (x * z + w * y); f.n[1] = 2 * (y * z - w * x); f.n[2] = 1 - 2 * (x * x + y * y);
  for (int a = 0; a < 3; ++a) f.p[a] = center[3 * k + a];
  for (int a = 0; a < 3; ++a) {
    const double r0 = cam.R[3 * a + 0], r1 = cam.R[3 * a + 1], r2 = cam.R[3 * a + 2];
    f.nc[a] = r0 * f.n[0] + r1 * f.n[1] + r2 * f.n[2];
    f.vxc[a] = r0 * f.vx[0] + r1 * f.vx[1] + r2 * f.vx[2];
    f.vyc[a] = r0 * f.vy[0] + r1 * f.vy[1] + r2 * f.vy[2];
  }
  const double t0 = cam.t[0], t1 = cam.t[1], t2 = cam.t[2];
  f.h = (f.p[0] * f.n[0] + f.p[1] * f.n[1] + f.p[2] * f.n[2]) + (t0 * f.nc[0] + t1 * f.nc[1] + t2 * f.nc[2]);
  f.pvx = (f.p[0] * f.vx[0] + f.p[1] * f.vx[1] + f.p[2] * f.vx[2]) + (t0 * f.vxc[0] + t1 * f.vxc[1] + t2 * f.vxc[2]);
  f.pvy = (f.p[0] * f.vy[0] + f.p[1] * f.vy[1] + f.p[2] * f.vy[2]) + (t0 * f.vyc[0] + t1 * f.vyc[1] + t2 * f.vyc[2]);
  return true;
}

}  // namespace ps
