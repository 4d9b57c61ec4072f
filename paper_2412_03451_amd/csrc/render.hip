// plane_render_fwd / plane_render_bwd: one wave64 workgroup per 8x8 pixel
// block ("item"); the block walks the depth-bound-sorted list of its tile.
//
// Exact per-ray order (Sec. 3.2: filter w >= tau, sort the survivors near to
// far, composite the first M).  Candidates arrive sorted by a lower bound of
// their depth over the tile.  Each lane keeps a small sorted buffer of pending
// hits and commits a hit only once the next candidate's bound exceeds its
// depth, so no later candidate can come before it.  A pending hit behind an
// opaque pending hit (w = 1) or beyond the first M is dropped.  A lane whose
// buffer would overflow finishes with an exact per-pixel selection scan
// resuming after its last committed hit.  Record data are wave-uniform and
// reach the SIMD through scalar loads; the ray-plane geometry runs in float64
// (full-rate FMA on CDNA), weights and compositing in float32.
//
// Backward: the block recomputes the same committed sequence, keeping for a
// chunk of C hits per lane (list position, w, transmittance T, c = gD t + gN.n)
// in LDS, plus the composite of the hits after the chunk.  A back-to-front
// walk gives dL/dw_j = T_j (c_j - S_{j+1}) with S_j = w_j c_j + (1 - w_j) S_{j+1}
// (no division by 1 - w).  The block then visits the chunk's candidates in
// list order (wave minimum of the lanes' next positions), forms per-pair
// gradients of 13 per-record accumulators and reduces them across the wave.
// Lists deeper than C hits take further recompute passes.  Partials per
// (pair, 8x8 block) are summed per record in a fixed order and chained to
// (center, quat, radii) by bwd_reduce_kernel.
#include <string.h>

#include <mutex>

#include "ps_internal.h"

using namespace ps;

int ps_check_ws(const ps_layout* L, const void* ws, const char* who);

namespace {

struct RenderArgs {
  const ps_slot* slots;
  int S, n_items;
  const Rec* recs;
  const ItemDesc* items;
  const Rec* recs_s;        // record copies in list order
  const uint64_t* keys;
  const uint32_t* emit;
  const int* rec_cnt;
  const int* rec_off;   // chunk-local (binning scan); add rbase[r / kScanChunk]
  const int* rbase;
  const ps_camera* cams;
  int n_cams;
  const float* lambda;
  float tau, z_near;
  double flog;              // filter_log(tau, mode)
  int M, mode, flags, two_sided;
  long long* counters;
  long long* diag;          // per-block statistics (flags bit 6)
  float* depth;
  float* normal;
  float* trans;      // optional: final transmittance per pixel
  int32_t* count;    // optional: committed hits per pixel
  // stored per-pixel lists [M][n_pixels] (the list-storing variant): list
  // position, a* and transmittance in front of each committed hit
  int32_t* lst_pos;
  float* lst_a;
  float* lst_T;
  int64_t lst_stride;
  const float* g_depth;
  const float* g_normal;
  float* partial;
  int max_sub;
  // reduction
  const float* center;
  const float* quat;
  int K;
  float* g_center;
  float* g_quat;
  float* g_radii;
  // the forward that forms the render loss (Eq. 14) of the pixels it renders:
  // gradients and per-8x8-block partial sums (null: plain forward)
  LossView loss;
  double* loss_part;
  int slots_sorted;   // plane ranges nondecreasing over the slots
  // work-queue counters of a persistent launch (8 per direction, one 128-byte
  // line each); the queue region until the launch, null in a launch of one
  // workgroup per item
  unsigned long long* queue;
  // plane_render_bwd_adam: the loss sums of the last forward with the loss,
  // formed by workgroups added to the per-plane reduction
  float* loss_out;
  const double* loss_in;
  // plane_render_bwd_adam, plane_render_step: the Adam update, applied by the
  // per-plane reduction to the gradients it forms (upd_m null: no update)
  float* upd_p[3];          // center, quat, radii, updated in place
  float* upd_m;
  float* upd_v;
  const int32_t* upd_step;
  float upd_lr[3], upd_b1, upd_b2, upd_eps, upd_rmin;
};

// LDS of the render workgroups, at namespace scope so that every access
// compiles to an LDS instruction (a pointer or reference kept in a struct
// would be a generic address): the staged candidates of a batch.
__shared__ StageLds g_stage;

struct ItemCtx {
  int b, e;          // list range in keys[]
  int sub;           // 8x8 block index inside the tile
  int slot;          // job of the block
  int ox, oy;        // pixel origin of the block
  int px, py;        // this lane's pixel
  bool inimg;
  int bx0, bx1, by0, by1;  // pixel box of the block (clipped to the image)
  double u, v, eps;  // pixel center, |den| threshold
  float du, dv;      // camera-frame ray (du, dv, 1)
  int64_t pix;       // index of the pixel in the depth array
  int64_t pix_off, HW;
};

// 0: block inside the image; 1: block entirely outside (partial tile); 2: bad camera
// Render item of workgroup b of n.  The dispatcher hands workgroups to the
// eight XCDs in turn (b runs on XCD b mod 8), and each XCD has its own L2;
// the 8x8 items of one tile are consecutive and read the same list records.
// Inside every aligned run of 32 workgroups, item 4 j + i goes to workgroup
// 8 i + (j mod 8) of the run: a group of four consecutive items shares one
// XCD, and the longest-first order of the items holds at a granularity of 32.
// The last n mod 32 workgroups map to themselves (a bijection either way).
__device__ inline int xcd_item(int b, int n) {
  if (b >= (n & ~31)) return b;
  const int k = b & 31;
  return (b & ~31) + ((k & 7) << 2) + (k >> 3);
}

// Issue priority of the wave for one item, by list length: the items with
// the longest lists set a launch's duration, and the waves sharing their SIMD
// (short items, mostly waiting on memory) lose little by yielding to them.
__device__ inline void item_priority(int n) {
  if (n >= 48)
    __builtin_amdgcn_s_setprio(3);
  else if (n >= 32)
    __builtin_amdgcn_s_setprio(2);
  else if (n >= 16)
    __builtin_amdgcn_s_setprio(1);
  else
    __builtin_amdgcn_s_setprio(0);
}

__device__ inline int item_setup(const RenderArgs& a, int item, ItemCtx& c) {
  const ItemDesc d = a.items[item];
  c.b = d.b;
  c.e = d.e;
  c.sub = d.sub;
  c.slot = d.slot;
  c.ox = d.ox;
  c.oy = d.oy;
  const int ox = d.ox, oy = d.oy, W = d.width, H = d.height;
  const int lane = threadIdx.x;
  c.px = ox + (lane & 7);
  c.py = oy + (lane >> 3);
  c.inimg = c.px < W && c.py < H;
  c.bx0 = ox; c.bx1 = min(ox + 7, W - 1);
  c.by0 = oy; c.by1 = min(oy + 7, H - 1);
  c.pix_off = d.pix_off;
  c.HW = (int64_t)W * H;
  c.pix = d.pix_off + (int64_t)c.py * W + c.px;
  if (d.cam < 0 || d.cam >= a.n_cams) return 2;
  const ps_camera& cam = a.cams[d.cam];
  c.u = c.px + 0.5;
  c.v = c.py + 0.5;
  const double du = (c.u - (double)cam.cx) / (double)cam.fx;
  const double dv = (c.v - (double)cam.cy) / (double)cam.fy;
  c.du = (float)du;
  c.dv = (float)dv;
  c.eps = 1e-12 * sqrt(du * du + dv * dv + 1.0);
  return (ox < W && oy < H) ? 0 : 1;
}

// Order key of a hit: the float32 depth's bits above the record index.  Hit
// depths are positive (t > z_near > 0), where the bits of a float order like
// the float, so one unsigned 64-bit comparison orders (t, record) as
// key_less does; depth bounds compare as bits(bound) << 32.
__device__ inline uint64_t hit_key(float t, int r) {
  return ((uint64_t)__float_as_uint(t) << 32) | (uint32_t)r;
}
__device__ inline float key_depth(uint64_t k) { return __uint_as_float((uint32_t)(k >> 32)); }
__device__ inline bool key_before(uint64_t k, float bound) {   // depth of k < bound (bound >= 0)
  return (uint32_t)(k >> 32) < __float_as_uint(bound);
}
constexpr uint64_t kNoKey = ~0ull;

// Sorted buffer of pending hits (ascending key), in registers.  Each entry
// keeps the float32 a* of the hit (weights are formed at commit time) and its
// list position; what the sink needs of the plane (its normal) is read back
// at commit time by list position, from the staged batch when the hit came
// from it.
template <int P>
struct Pending {
  uint64_t k[P];
  float a[P];
  int pos[P];
  int n;
  uint64_t ok;   // key of the opaque pending hit, kNoKey if none
  uint64_t lk;   // key of the last pending hit, 0 if none

  __device__ void reset() {
    n = 0;
    ok = kNoKey;
    lk = 0;
  }

  // Keep the `cap` nearest hits (cap = hits still allowed by M, or fewer).
  // false: the buffer is full and the hit may still be among the nearest cap.
  // Selects only, no per-lane branches: every entry is rewritten from
  // itself, its lower neighbour or the new hit.
  __device__ bool insert(uint64_t nk, float na, bool opq, int npos, int cap) {
    const bool full = n >= cap;
    // dropped: behind an opaque pending hit, or not among the nearest cap
    const bool drop = (ok < nk) || (full && (n == 0 || !(nk < lk)));
    const bool ovf = !drop && !full && n == P;
    const bool put = !drop && !ovf;
    // a full buffer gives up its last entry (an opaque hit is always the last)
    const int m = (put && full) ? n - 1 : n;
    ok = (put && full) ? kNoKey : ok;
    // place of the new hit: the number of entries below it (keys are unique)
    int at = 0;
#pragma unroll
    for (int i = 0; i < P; ++i) at += (i < m && k[i] < nk) ? 1 : 0;
    // entries at..m-1 move up one place (from the top, so each reads its
    // lower neighbour before that one moves)
#pragma unroll
    for (int i = P - 1; i > 0; --i) {
      const bool up = put && i > at && i <= m;
      k[i] = up ? k[i - 1] : k[i];
      a[i] = up ? a[i - 1] : a[i];
      pos[i] = up ? pos[i - 1] : pos[i];
    }
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const bool here = put && i == at;
      k[i] = here ? nk : k[i];
      a[i] = here ? na : a[i];
      pos[i] = here ? npos : pos[i];
    }
    n = put ? m + 1 : n;
    // everything behind an opaque hit is hidden
    n = (put && opq) ? at + 1 : n;
    ok = (put && opq) ? nk : ok;
#pragma unroll
    for (int i = 0; i < P; ++i) lk = (put && i == n - 1) ? k[i] : lk;
    return !ovf;
  }

  __device__ void pop(uint64_t& fk, float& fa, int& fpos) {
    fk = k[0]; fa = a[0]; fpos = pos[0];
#pragma unroll
    for (int i = 0; i + 1 < P; ++i) {
      k[i] = k[i + 1]; a[i] = a[i + 1]; pos[i] = pos[i + 1];
    }
    n -= 1;
    if (n == 0) { lk = 0; ok = kNoKey; }
  }
};

// Stage the batch [base, base + kBatch) of the tile list: each of the first
// kBatch lanes fetches one list entry (its key and the 128-byte record copy: coalesced, one memory
// latency per batch) and stores the record head in LDS if the record's pixel
// box overlaps the 8x8 block; the backward also keeps the in-plane offsets and
// the emit index.  Returns the mask of overlapping candidates.
template <bool BWD>
__device__ inline uint64_t stage_batch(const RenderArgs& a, const ItemCtx& c, int base) {
  StageLds& S = g_stage;
  const int lane = threadIdx.x;
  const int i = base + lane;
  bool ov = false;
  if (lane < kBatch && i < c.e) {
    const uint64_t key = a.keys[i];
    const float4* src = reinterpret_cast<const float4*>(&a.recs_s[i]);
    const float4 h0 = src[0], h1 = src[1], h2 = src[2], h3 = src[3];
    const float4 h4 = src[4], h5 = src[5], h6 = src[6], h7 = src[7];
    const uint32_t em = BWD ? a.emit[i] : 0u;
    const uint32_t b0 = __float_as_uint(h7.x), b1 = __float_as_uint(h7.y);
    const int px0 = (int16_t)(b0 & 0xffffu), py0 = (int16_t)(b0 >> 16);
    const int px1 = (int16_t)(b1 & 0xffffu), py1 = (int16_t)(b1 >> 16);
    ov = !(px1 < c.bx0 || px0 > c.bx1 || py1 < c.by0 || py0 > c.by1);
    if (ov) {
      S.head[0][lane] = h0; S.head[1][lane] = h1; S.head[2][lane] = h2; S.head[3][lane] = h3;
      S.head[4][lane] = h4; S.head[5][lane] = h5; S.head[6][lane] = h6;
      if (BWD) S.pv[lane] = make_float2(h7.z, h7.w);
    }
    if (BWD) S.em[lane] = em;
    S.tlb[lane] = __uint_as_float((uint32_t)(key >> 32));
    S.rec[lane] = (int)(uint32_t)key;
  }
  const uint64_t m = ballot(ov);
  __syncthreads();
  return m;
}

__device__ inline double dbl(float lo, float hi) {
  return __hiloint2double(__float_as_int(hi), __float_as_int(lo));
}

__device__ inline void staged(const StageLds& S, int j, RecHead& rec, float n[3]) {
  const float4 h0 = S.head[0][j], h1 = S.head[1][j], h2 = S.head[2][j], h3 = S.head[3][j];
  const float4 h4 = S.head[4][j], h5 = S.head[5][j], h6 = S.head[6][j];
  rec.D0 = dbl(h0.x, h0.y); rec.Du = dbl(h0.z, h0.w);
  rec.Dv = dbl(h1.x, h1.y); rec.X0 = dbl(h1.z, h1.w);
  rec.Xu = dbl(h2.x, h2.y); rec.Xv = dbl(h2.z, h2.w);
  rec.Y0 = dbl(h3.x, h3.y); rec.Yu = dbl(h3.z, h3.w);
  rec.Yv = dbl(h4.x, h4.y); rec.h = dbl(h4.z, h4.w);
  rec.rxp = h5.x; rec.rxm = h5.y; rec.ryp = h5.z; rec.rym = h5.w;
  n[0] = h6.x; n[1] = h6.y; n[2] = h6.z;
}

// Normal of the candidate at list position pos (relative to the item's list):
// from the staged batch starting at list index sb when it is there, else
// from the record copy in memory (a hit kept pending across batches).  A
// list of at most one batch is staged whole (sb = c.b): LDS only.
__device__ inline void cand_normal(const RenderArgs& a, const ItemCtx& c, int sb, int pos, float n[3]) {
  float4 h;
  if (c.e - c.b <= kBatch) {
    h = g_stage.head[6][pos];
  } else {
    const int j = c.b + pos - sb;
    const bool in = j >= 0 && j < kBatch;
    h = g_stage.head[6][in ? j : 0];
    if (!in) {
      // a volatile read: kept apart from the LDS reads above (merged, both
      // would become generic-address loads)
      const volatile float* g = reinterpret_cast<const volatile float*>(&a.recs_s[c.b + pos]) + 24;
      h.x = g[0]; h.y = g[1]; h.z = g[2];
    }
  }
  n[0] = h.x; n[1] = h.y; n[2] = h.z;
}

// Pop the nearest pending hit and hand it to the sink with its payload.
template <int P, class Sink>
__device__ __forceinline__ void commit_next(const RenderArgs& a, const ItemCtx& c, int sb, Pending<P>& pd,
                                            Sink& sink, uint64_t& lk) {
  uint64_t fk; float fa; int fp;
  pd.pop(fk, fa, fp);
  const float ft = key_depth(fk);
  float nrm[3], pl[Sink::NP];
  cand_normal(a, c, sb, fp, nrm);
  sink.payload(ft, nrm, pl);
  sink.commit(ft, fa, fp, pl);
  lk = fk;
}

// Commit the pending hits nearer than `bound` (no later candidate can precede them).
template <int P, class Sink>
__device__ __forceinline__ void drain(const RenderArgs& a, const ItemCtx& c, int sb, Pending<P>& pd, Sink& sink,
                                      int M, float bound, bool& done, uint64_t& lk) {
  bool want = !done && pd.n > 0 && key_before(pd.k[0], bound);
  if (ballot(want)) {
    while (want) {
      commit_next(a, c, sb, pd, sink, lk);
      if (sink.finished(M)) { done = true; break; }
      want = pd.n > 0 && key_before(pd.k[0], bound);
    }
  }
}

// Walk the tile list of one 8x8 block and hand every committed hit, in exact
// per-ray order, to sink.commit(t, a*, list position, payload), the payload
// formed by sink.payload(t, normal of the plane).
// Returns whether this lane took the exact fallback (its buffer overflowed).
template <int P, bool GAUSS, class Sink>
__device__ __forceinline__ bool walk(const RenderArgs& a, const ItemCtx& c, Sink& sink, float lam5,
                                     double delta, long long& evals, long long& steps) {
  Pending<P> pd;
  pd.reset();
  bool slow = (a.flags & 1) && c.inimg;
  bool done = !c.inimg || slow || sink.finished(a.M);
  uint64_t lk = 0;   // key of the last committed hit
  StageLds& S = g_stage;
  bool stop = ballot(!done) == 0;
  for (int base = c.b; base < c.e && !stop; base += kBatch) {
    uint64_t ovm = stage_batch<Sink::BWD>(a, c, base);
    // bound of every candidate after this batch
    const float tlb_after =
        (base + kBatch < c.e) ? __uint_as_float((uint32_t)(a.keys[base + kBatch] >> 32)) : INFINITY;
    while (ovm) {
      const int j = __ffsll((unsigned long long)ovm) - 1;
      ovm &= ovm - 1;
      ++steps;
      // only candidates overlapping this block can hit its pixels, so the next
      // one's bound (or the bound after the batch) limits every remaining hit
      const float tlb_next = ovm ? S.tlb[__ffsll((unsigned long long)ovm) - 1] : tlb_after;
      RecHead rec;
      float nrm[3];
      staged(S, j, rec, nrm);
      const int ri = S.rec[j];
      evals += __popcll(ballot(!done));
      const PairGeom g = eval_pair<GAUSS>(rec, c.u, c.v, c.eps, (double)a.z_near, delta);
      const bool hit = g.ok && !done;
      const float t32 = (float)g.t;
      const float a32 = (float)g.a;
      // nothing pending and no later candidate can come before it: commit
      // now (what inserting and draining to tlb_next would do)
      const bool now = hit && pd.n == 0 && t32 < tlb_next;
      if (ballot(now)) {
        if (now) {
          float pl[Sink::NP];
          sink.payload(t32, nrm, pl);
          sink.commit(t32, a32, base + j - c.b, pl);
          lk = hit_key(t32, ri);
          if (sink.finished(a.M)) done = true;
        }
      }
      const bool ins = hit && !now;
      if (ballot(ins)) {
        if (ins) {
          if (!pd.insert(hit_key(t32, ri), a32, a.mode == 0 && a32 >= 0.f, base + j - c.b, a.M - sink.count)) {
            slow = true;
            done = true;
          }
        }
      }
      drain(a, c, base, pd, sink, a.M, tlb_next, done, lk);
      if (ballot(!done) == 0) {
        stop = true;
        break;
      }
    }
    // pending hits below the bound of everything after this batch
    if (!stop) {
      drain(a, c, base, pd, sink, a.M, tlb_after, done, lk);
      stop = ballot(!done) == 0;
    }
    __syncthreads();
  }
  const uint64_t slow_mask = ballot(slow);
  const bool took_fallback = slow;
  if (slow_mask && threadIdx.x == 0)
    atomicAdd((unsigned long long*)&a.counters[C_SLOW], (unsigned long long)__popcll(slow_mask));
  // Exact continuation for lanes whose buffer overflowed: rounds that each
  // collect the P nearest hits after the last committed one in one scan of
  // the list (a candidate whose bound exceeds the P-th collected depth cannot
  // contribute, so the scan stops once every such lane is saturated), then
  // commit them in order.  At most ceil(M / P) rounds.
  while (ballot(slow && !sink.finished(a.M))) {
    const bool act = slow && !sink.finished(a.M);
    pd.reset();
    const int cap = min(P, a.M - sink.count);
    bool stop2 = false;
    int sb = c.b;   // the batch left staged in LDS
    for (int base = c.b; base < c.e && !stop2; base += kBatch) {
      uint64_t ovm = stage_batch<Sink::BWD>(a, c, base);
      sb = base;
      while (ovm) {
        const int j = __ffsll((unsigned long long)ovm) - 1;
        ovm &= ovm - 1;
        const float tj = S.tlb[j];
        const bool sat = (pd.n >= cap || pd.ok != kNoKey) && pd.n > 0 && key_before(pd.lk, tj);
        const bool need = act && !sat;
        if (ballot(need) == 0) {
          stop2 = true;
          break;
        }
        ++steps;
        RecHead rec;
        float nrm[3];
        staged(S, j, rec, nrm);
        const int ri = S.rec[j];
        evals += __popcll(ballot(need));
        const PairGeom g = eval_pair<GAUSS>(rec, c.u, c.v, c.eps, (double)a.z_near, delta);
        if (need && g.ok) {
          const float t32 = (float)g.t;
          const float a32 = (float)g.a;
          const uint64_t nk = hit_key(t32, ri);
          if (lk < nk) pd.insert(nk, a32, a.mode == 0 && a32 >= 0.f, base + j - c.b, cap);
        }
      }
      __syncthreads();
    }
    if (act) {
      const bool exhausted = pd.n < cap && pd.ok == kNoKey;
      while (pd.n > 0 && !sink.finished(a.M)) commit_next(a, c, sb, pd, sink, lk);
      if (exhausted) slow = false;
    }
  }
  return took_fallback;
}

// ------------------------------------------------------------------ forward
struct FwdSink {
  static constexpr int NP = 3;   // payload: rendered normal of the hit
  static constexpr bool BWD = false;
  float T, D, N0, N1, N2;
  int count;
  float lam5;
  int mode;
  const RenderArgs* args;   // list storage (lst_pos non-null) and the lane's pixel
  int64_t pix;
  __device__ bool finished(int M) const { return T == 0.f || count >= M; }
  __device__ void payload(float, const float n[3], float* pl) const {
    pl[0] = n[0]; pl[1] = n[1]; pl[2] = n[2];
  }
  __device__ void commit(float t, float as, int pos, const float* n) {
    if (args->lst_pos) {
      const int64_t o = (int64_t)count * args->lst_stride + pix;
      args->lst_pos[o] = pos;
      args->lst_a[o] = as;
      args->lst_T[o] = T;
    }
    float omw;
    const float w = splat_weight(as, lam5, mode, omw);
    const float Tw = T * w;
    D = fmaf(Tw, t, D);                 // Eq. 11
    N0 = fmaf(Tw, n[0], N0);            // Eq. 12
    N1 = fmaf(Tw, n[1], N1);
    N2 = fmaf(Tw, n[2], N2);
    T = T * omw;                        // Eq. 13
    ++count;
  }
};

// The render loss of this 8x8 block's pixels (the loss kernel's arithmetic)
// and the block's partial sums, stored where the loss kernel stores them: at
// the job's first item plus the block's index in tile order.
// g (optional): the pixel's loss gradient (zeros without a pixel).
__device__ void block_loss(const RenderArgs& a, const ItemCtx& c, const ps_slot& sl, const LossTargets& tg,
                           bool pix_on, float D, float N0, float N1, float N2, float* g = nullptr) {
  double l[4] = {0, 0, 0, 0};
  if (g) g[0] = g[1] = g[2] = g[3] = 0.f;
  if (pix_on) {
    const float N[3] = {N0, N1, N2};
    loss_apply(a.loss, tg, D, N, l, g);
  }
  for (int q = 0; q < 4; ++q) l[q] = wave_sum_double(l[q]);
  if (threadIdx.x == 0) {
    const int sub_per = (sl.tile_w >> 3) * (sl.tile_h >> 3);
    const int tile = (c.oy / sl.tile_h) * sl.tiles_x + c.ox / sl.tile_w;
    double* o = a.loss_part + 4 * ((size_t)sl.item_begin + (size_t)tile * sub_per + c.sub);
    o[0] = l[0]; o[1] = l[1]; o[2] = l[2]; o[3] = l[3];
  }
}

template <int P, bool GAUSS>
__device__ __forceinline__ void fwd_item(const RenderArgs& a, int item) {
  const bool diag = a.flags & kFlagDiag;
  const uint64_t t_start = diag ? wall_clock64() : 0;
  long long* dg = a.diag + (size_t)item * D_NUM;
  if (diag && threadIdx.x < D_BWD_SETUP) dg[threadIdx.x] = 0;
  ItemCtx c;
  const int st = item_setup(a, item, c);
  // the loss targets of the pixel are read now; their latency overlaps the walk
  ps_slot sl;
  LossTargets tg;
  if (a.loss_part) {
    sl = a.slots[c.slot];
    tg = loss_targets(a.loss, sl, c.inimg ? c.px : 0, c.inimg ? c.py : 0);
  }
  if (st != 0) {
    // no render here; the loss still needs the block's partials (zero) and,
    // for a camera out of range, zero gradients
    if (a.loss_part) block_loss(a, c, sl, tg, st == 2 && c.inimg, 0.f, 0.f, 0.f, 0.f);
    return;
  }
  item_priority(c.e - c.b);
  const float lam = a.lambda[0];
  const float lam5 = 5.f * lam;
  const double delta = fringe_margin((double)lam, a.flog, a.mode);
  FwdSink s{1.f, 0.f, 0.f, 0.f, 0.f, 0, lam5, a.mode, &a, c.pix};
  long long evals = 0, steps = 0;
  const bool took_fallback = walk<P, GAUSS>(a, c, s, lam5, delta, evals, steps);
  if (diag) {
    int commits = s.count;
    commits = wave_allreduce(commits, [](int x, int y) { return x + y; });
    if (threadIdx.x == 0) {
      dg[D_EVALS] = evals;
      dg[D_COMMITS] = commits;
      dg[D_STEPS] = steps;
      dg[D_FWD_TICKS] = (long long)(wall_clock64() - t_start);
    }
  }
  if (c.inimg) {
    a.depth[c.pix] = s.D;
    if (a.trans) a.trans[c.pix] = s.T;
    if (a.count) a.count[c.pix] = s.count + ((a.flags & kFlagPathDiag) && took_fallback ? 256 : 0);
    const int64_t nb = 3 * c.pix_off + (c.pix - c.pix_off);
    a.normal[nb] = s.N0;
    a.normal[nb + c.HW] = s.N1;
    a.normal[nb + 2 * c.HW] = s.N2;
  }
  if (a.loss_part) block_loss(a, c, sl, tg, c.inimg, s.D, s.N0, s.N1, s.N2);
}

// Persistent launches (a batch with more 8x8 items than the chip holds
// resident): the grid is the resident capacity and every workgroup claims
// work from an atomic queue until none remains.  The unit of a claim is a
// group of four consecutive items (the 8x8 blocks of one 16x16 tile read the
// same list), so a claim costs one atomic per four items.  Groups keep the
// longest-first order and are dealt to eight streams in turn, stream x for
// the workgroups the dispatcher places on XCD x (b mod 8), which keeps a
// tile's list in one L2 as xcd_item does.  Each stream's counter has a
// 128-byte line of its own: the atomics of one stream do not wait behind
// those of the others.  A workgroup whose stream is empty moves to streams
// that a plain read shows are not (no atomic on an empty stream).  A small
// kernel after the launch clears the counters.
constexpr int kQueueStride = 16;   // u64 words between stream counters (128 bytes)

__device__ inline int claim_group(unsigned long long* cnt, int n_groups, int& stream) {
  for (int tries = 0; tries < 8; ++tries) {
    const int x = (stream + tries) & 7;
    // groups of stream x: x, x + 8, ...; its counter counts claims
    const int per = n_groups > x ? (n_groups - x + 7) >> 3 : 0;
    if (__hip_atomic_load(&cnt[x * kQueueStride], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >=
        (unsigned long long)per)
      continue;
    unsigned long long l = 0;
    if (threadIdx.x == 0) l = atomicAdd(&cnt[x * kQueueStride], 1ull);
    l = __shfl(l, 0, 64);
    if (l < (unsigned long long)per) {
      stream = x;
      return x + 8 * (int)l;
    }
  }
  return -1;
}

__global__ void queue_reset_kernel(unsigned long long* cnt) {
  if (threadIdx.x < 8) cnt[threadIdx.x * kQueueStride] = 0ull;
}

template <int P, bool GAUSS, bool PERSIST>
__global__ __launch_bounds__(64) void render_fwd_kernel(RenderArgs a) {
  if (a.counters[C_OVERFLOW]) return;
  if (!PERSIST) {
    fwd_item<P, GAUSS>(a, xcd_item(blockIdx.x, gridDim.x));
    return;
  }
  const int n_groups = (a.n_items + 3) >> 2;
  int stream = blockIdx.x & 7;
  for (int g = claim_group(a.queue, n_groups, stream); g >= 0; g = claim_group(a.queue, n_groups, stream)) {
    for (int item = 4 * g; item < min(4 * g + 4, a.n_items); ++item) {
      fwd_item<P, GAUSS>(a, item);
      __syncthreads();
    }
  }
}

// ------------------------------------------------------------------ backward
constexpr int kChunk = 8;    // hits per lane kept in LDS per recompute pass
constexpr int kPrioList = 256;   // tile lists from this length get the raised wave priority

struct BwdLds {
  int16_t pos[kChunk][64];   // list positions (< 4096)
  float a[kChunk][64];    // a* of the hit
  float T[kChunk][64];    // transmittance in front of the hit
  float cg[kChunk][64];   // c_j, then dL/dw_j after the back-to-front walk
  int16_t hpos[kMaxM][64];  // list positions of the committed hits, in commit order
  int gpos[64];           // a group of candidates of the gradient pass: list positions, ascending
  uint32_t vis[kBigSort / 32];  // list positions visited by the first gradient pass (lists up to kBigSort)
};
__shared__ BwdLds g_bwd;

// Sum 16 per-lane values over the wave by recursive halving: each exchange
// step sends half of the values still held (permlane swaps across the wave
// halves and the 16-lane rows, then DPP mirrors inside the rows, then quad
// permutes), 8 + 4 + 2 + 1 + 2 exchanges in all, none through LDS.  On return
// lane 4 q + r (r < 4) holds the total of value q, summed in a fixed order;
// the four lanes of a quad hold the same bits.
__device__ __forceinline__ float wave_sum16(float (&v)[16]) {
  const int lane = threadIdx.x;
  // lane ^ 32: lanes 0-31 keep values 0-7, lanes 32-63 values 8-15
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[i]), __float_as_uint(v[i + 8]), false, false);
    v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  // lane ^ 16: lanes with bit 4 clear keep the first 4 of their 8, the others the last 4
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[i]), __float_as_uint(v[i + 4]), false, false);
    v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  // lane ^ 15 (row mirror): bit 3 picks 2 of the 4
  const bool u8 = lane & 8;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const float send = u8 ? v[i] : v[i + 2];
    const float keep = u8 ? v[i + 2] : v[i];
    v[i] = keep + dpp_float<kDppMirror16>(send);
  }
  // lane ^ 7 (half-row mirror): bit 2 picks 1 of the 2
  const bool u4 = lane & 4;
  const float send = u4 ? v[0] : v[1];
  const float keep = u4 ? v[1] : v[0];
  float r = keep + dpp_float<kDppMirror8>(send);
  r += dpp_float<kDppXor2>(r);
  r += dpp_float<kDppXor1>(r);
  return r;
}

static_assert(3 * kChunk < kMaxM && 4 * kChunk >= kMaxM, "chunk starts: at most four chunks of a list of M hits");

struct BwdSink {
  static constexpr int NP = 1;   // payload: c = gD t + gN . n of the hit
  static constexpr bool BWD = true;
  float T;
  int count;
  int c0;
  float Tb1, Tb2, Tb3;   // transmittance in front of hits 8, 16, 24 (chunk starts)
  float gD, gN0, gN1, gN2;
  float lam5;
  int mode;
  __device__ bool finished(int M) const { return T == 0.f || count >= M; }
  __device__ void payload(float t, const float n[3], float* pl) const {
    // explicit fma chain: the same bits whichever path commits the hit
    pl[0] = fmaf(gD, t, fmaf(gN0, n[0], fmaf(gN1, n[1], gN2 * n[2])));
  }
  __device__ void commit(float t, float as, int pos, const float* pl) {
    float omw;
    const float w = splat_weight(as, lam5, mode, omw);
    const float cv = pl[0];
    const int j = count - c0;
    const int lane = threadIdx.x;
    BwdLds& L = g_bwd;
    L.hpos[count][lane] = (int16_t)pos;
    if (j >= 0 && j < kChunk) {
      L.pos[j][lane] = pos;
      L.a[j][lane] = as;
      L.T[j][lane] = T;
      L.cg[j][lane] = cv;
    }
    if (count == kChunk) Tb1 = T;
    if (count == 2 * kChunk) Tb2 = T;
    if (count == 3 * kChunk) Tb3 = T;
    T = T * omw;
    ++count;
  }
};

// The fused forward-and-backward walk of the fitting step: composites depth
// and normal like the forward (the same arithmetic, so the same bits) and
// records what the backward needs of every committed hit: its list position
// and the transmittance at each chunk start; and, in chunk slots taken
// cyclically (hit j in slot j mod kChunk), a*, the transmittance in front of
// the hit and its depth, so that the pixel's last chunk is in LDS when the
// walk ends.  The per-hit values of the gradient pass wait for the pixel's
// loss gradient, which exists only once the pixel is composited: they are
// formed from the depth and the plane's normal then, for the last chunk
// (the first one the backward processes); the other chunks are committed
// again from the positions.
struct FwdBwdSink {
  static constexpr int NP = 3;   // payload: rendered normal of the hit
  static constexpr bool BWD = true;
  float T, D, N0, N1, N2;
  int count;
  float Tb1, Tb2, Tb3;   // transmittance in front of hits 8, 16, 24 (chunk starts)
  float lam5;
  int mode;
  __device__ bool finished(int M) const { return T == 0.f || count >= M; }
  __device__ void payload(float, const float n[3], float* pl) const {
    pl[0] = n[0]; pl[1] = n[1]; pl[2] = n[2];
  }
  __device__ void commit(float t, float as, int pos, const float* n) {
    BwdLds& L = g_bwd;
    const int lane = threadIdx.x;
    L.hpos[count][lane] = (int16_t)pos;
    const int j = count % kChunk;
    L.pos[j][lane] = pos;
    L.a[j][lane] = as;
    L.T[j][lane] = T;
    L.cg[j][lane] = t;   // the depth, until the loss gradient exists
    if (count == kChunk) Tb1 = T;
    if (count == 2 * kChunk) Tb2 = T;
    if (count == 3 * kChunk) Tb3 = T;
    float omw;
    const float w = splat_weight(as, lam5, mode, omw);
    const float Tw = T * w;
    D = fmaf(Tw, t, D);                 // Eq. 11
    N0 = fmaf(Tw, n[0], N0);            // Eq. 12
    N1 = fmaf(Tw, n[1], N1);
    N2 = fmaf(Tw, n[2], N2);
    T = T * omw;                        // Eq. 13
    ++count;
  }
};

// Commit again, in the same order, the hits that the first pass's walk
// committed (their list positions are in L.hpos): the same evaluation of the
// same records gives the same bits, without walking the list again.
// Only the hits [j0, min(j1, hits)) are committed; s starts at hit j0 (its
// count and the transmittance in front of that hit).
__device__ inline void replay(const RenderArgs& a, const ItemCtx& c, BwdSink& s, int j0, int j1, int hits,
                              bool one_batch, double delta) {
  const int jmax = min(j1, wave_max_int(hits));
  const int lane = threadIdx.x;
  for (int j = j0; j < jmax; ++j) {
    if (j < hits) {
      const int pos = g_bwd.hpos[j][lane];
      RecHead rec;
      float nrm[3];
      if (one_batch) {
        staged(g_stage, pos, rec, nrm);
      } else {
        const float4* src = reinterpret_cast<const float4*>(&a.recs_s[c.b + pos]);
        const float4 h0 = src[0], h1 = src[1], h2 = src[2], h3 = src[3], h4 = src[4], h5 = src[5], h6 = src[6];
        rec.D0 = dbl(h0.x, h0.y); rec.Du = dbl(h0.z, h0.w);
        rec.Dv = dbl(h1.x, h1.y); rec.X0 = dbl(h1.z, h1.w);
        rec.Xu = dbl(h2.x, h2.y); rec.Xv = dbl(h2.z, h2.w);
        rec.Y0 = dbl(h3.x, h3.y); rec.Yu = dbl(h3.z, h3.w);
        rec.Yv = dbl(h4.x, h4.y); rec.h = dbl(h4.z, h4.w);
        rec.rxp = h5.x; rec.rxm = h5.y; rec.ryp = h5.z; rec.rym = h5.w;
        nrm[0] = h6.x; nrm[1] = h6.y; nrm[2] = h6.z;
      }
      const PairGeom g = eval_pair_mode(rec, c.u, c.v, c.eps, (double)a.z_near, delta, a.mode);
      const float t32 = (float)g.t;
      const float a32 = (float)g.a;
      float pl[1];
      s.payload(t32, nrm, pl);
      s.commit(t32, a32, pos, pl);
    }
  }
}

// The list-storing variant: commit the hits the forward stored for this
// pixel (list position and a*), recomputing only the depth and normal of each.
__device__ inline void load_lists(const RenderArgs& a, const ItemCtx& c, BwdSink& s, int hits, bool one_batch,
                                  double delta) {
  const int jmax = wave_max_int(hits);
  for (int j = 0; j < jmax; ++j) {
    if (j < hits) {
      const int64_t o = (int64_t)j * a.lst_stride + c.pix;
      const int pos = a.lst_pos[o];
      const float as = a.lst_a[o];
      RecHead rec;
      float nrm[3];
      if (one_batch) {
        staged(g_stage, pos, rec, nrm);
      } else {
        const float4* src = reinterpret_cast<const float4*>(&a.recs_s[c.b + pos]);
        const float4 h0 = src[0], h1 = src[1], h2 = src[2], h3 = src[3], h4 = src[4], h5 = src[5], h6 = src[6];
        rec.D0 = dbl(h0.x, h0.y); rec.Du = dbl(h0.z, h0.w);
        rec.Dv = dbl(h1.x, h1.y); rec.X0 = dbl(h1.z, h1.w);
        rec.Xu = dbl(h2.x, h2.y); rec.Xv = dbl(h2.z, h2.w);
        rec.Y0 = dbl(h3.x, h3.y); rec.Yu = dbl(h3.z, h3.w);
        rec.Yv = dbl(h4.x, h4.y); rec.h = dbl(h4.z, h4.w);
        rec.rxp = h5.x; rec.rxm = h5.y; rec.ryp = h5.z; rec.rym = h5.w;
        nrm[0] = h6.x; nrm[1] = h6.y; nrm[2] = h6.z;
      }
      const PairGeom g = eval_pair_mode(rec, c.u, c.v, c.eps, (double)a.z_near, delta, a.mode);
      float pl[1];
      s.payload((float)g.t, nrm, pl);
      s.commit((float)g.t, as, pos, pl);
    }
  }
}

__device__ inline void zero_row(const RenderArgs& a, uint32_t em, int sub) {
  float4* row = (float4*)(a.partial + ((size_t)em * a.max_sub + sub) * 16);
  const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
  row[0] = z; row[1] = z; row[2] = z; row[3] = z;
}

// Partial rows: every (list entry, 8x8 block) row of the tile is written by
// its block, exactly once in the first pass (the gradient of a candidate the
// block hits, zeros otherwise); further passes add to it.
//
// FUSED (the fitting step): the same block's forward and loss come first, in
// the same walk (FwdBwdSink): depth and normal are written, the loss of
// Eq. 14 is formed per pixel (the forward-with-loss arithmetic: the same
// partials and loss gradients), and the gradient passes take the pixel's
// loss gradient from registers.  Every chunk, the first too, is committed
// again from the recorded positions: the same bits as the two separate calls.
template <int P, bool GAUSS, bool FUSED>
__device__ __forceinline__ void bwd_item(const RenderArgs& a, int item) {
  BwdLds& L = g_bwd;
  StageLds& stage = g_stage;
  const bool diag = a.flags & kFlagDiag;
  uint64_t tk = diag ? wall_clock64() : 0;
  unsigned long long ph[4] = {0, 0, 0, 0}, ncand = 0, ngrp = 0;
  auto mark = [&](int i) {
    if (diag) {
      const uint64_t now = wall_clock64();
      ph[i] += now - tk;
      tk = now;
    }
  };
  long long* dg = a.diag + (size_t)item * D_NUM;
  if (diag && threadIdx.x >= D_BWD_SETUP && threadIdx.x <= D_BWD_TICKS) dg[threadIdx.x] = 0;
  ItemCtx c;
  const int st = item_setup(a, item, c);
  // the loss targets of the pixel are read now; their latency overlaps the walk
  ps_slot sl;
  LossTargets tg;
  if (FUSED) {
    sl = a.slots[c.slot];
    tg = loss_targets(a.loss, sl, c.inimg ? c.px : 0, c.inimg ? c.py : 0);
    // no render here: the block's loss partials (zero) and, for a camera out
    // of range, zero loss gradients
    if (st != 0) block_loss(a, c, sl, tg, st == 2 && c.inimg, 0.f, 0.f, 0.f, 0.f);
  }
  if (st == 2) return;
  const int lane = threadIdx.x;
  const int n = c.e - c.b;
  // the blocks of long tile lists set the launch's length: their waves win
  // the SIMD's instruction arbitration over the short ones sharing it (issue
  // order only, the arithmetic is unchanged; on the 640x480 room 0.1621 ->
  // 0.1606 ms per step, the 64-room batch unchanged)
  if (n >= kPrioList) __builtin_amdgcn_s_setprio(2);
  else __builtin_amdgcn_s_setprio(0);
  if (st == 1) {   // block outside the image (partial tile): zero rows
    for (int i = lane; i < n; i += 64) zero_row(a, a.emit[c.b + i], c.sub);
    return;
  }
  item_priority(n);
  // a list longer than the visit bitmask covers: clear all of its rows first,
  // then every pass adds
  const bool big = n > kBigSort;
  if (big) {
    for (int i = lane; i < n; i += 64) zero_row(a, a.emit[c.b + i], c.sub);
    __threadfence_block();
  }
  for (int i = lane; i < kBigSort / 32; i += 64) L.vis[i] = 0u;
  const float lam = a.lambda[0];
  const float lam5 = 5.f * lam;
  const double delta = fringe_margin((double)lam, a.flog, a.mode);
  float gD = 0.f, gN0 = 0.f, gN1 = 0.f, gN2 = 0.f;
  if (!FUSED && c.inimg) {
    gD = a.g_depth[c.pix];
    const int64_t nb = 3 * c.pix_off + (c.pix - c.pix_off);
    gN0 = a.g_normal[nb];
    gN1 = a.g_normal[nb + c.HW];
    gN2 = a.g_normal[nb + 2 * c.HW];
  }
  // a list of at most one batch stays staged in LDS after the walk
  const bool one_batch = n <= kBatch;
  mark(0);
  // The walk commits every hit once, keeping the first chunk of kChunk hits
  // per lane in LDS, every hit's list position and the transmittance at each
  // chunk start.  Chunks are then processed last to first: a chunk after the
  // first is committed again from its list positions (its transmittance
  // restored, the same bits as the walk), the back-to-front recurrence
  // carries the composite of everything behind it, and its candidates get
  // their gradients.  Each hit is evaluated once after the walk.
  int hits = 0;   // hits committed by the walk
  BwdSink s{1.f, 0, 0, 1.f, 1.f, 1.f, gD, gN0, gN1, gN2, lam5, a.mode};
  {
    long long evals = 0, steps = 0;
    if (FUSED) {
      FwdBwdSink f{1.f, 0.f, 0.f, 0.f, 0.f, 0, 1.f, 1.f, 1.f, lam5, a.mode};
      walk<P, GAUSS>(a, c, f, lam5, delta, evals, steps);
      hits = f.count;
      s.Tb1 = f.Tb1; s.Tb2 = f.Tb2; s.Tb3 = f.Tb3;
      if (c.inimg && a.depth) {
        a.depth[c.pix] = f.D;
        const int64_t nb = 3 * c.pix_off + (c.pix - c.pix_off);
        a.normal[nb] = f.N0;
        a.normal[nb + c.HW] = f.N1;
        a.normal[nb + 2 * c.HW] = f.N2;
      }
      float g[4];
      block_loss(a, c, sl, tg, c.inimg, f.D, f.N0, f.N1, f.N2, g);
      if (c.inimg) {
        gD = g[0]; gN0 = g[1]; gN1 = g[2]; gN2 = g[3];
      }
      // the per-hit values c_j of each pixel's last chunk now
      // (BwdSink::payload's arithmetic); the backward's first pass takes
      // them without committing that chunk again (a lane whose last chunk is
      // not the block's last gets its chunks committed again later)
      for (int j = hits > 0 ? (hits - 1) / kChunk * kChunk : 0; j < hits; ++j) {
        const int q = j % kChunk;
        float nrm[3];
        cand_normal(a, c, c.e, L.pos[q][lane], nrm);
        L.cg[q][lane] = fmaf(gD, L.cg[q][lane], fmaf(gN0, nrm[0], fmaf(gN1, nrm[1], gN2 * nrm[2])));
      }
    } else if (a.lst_pos) {
      // no walk: stage the first batch here (record heads, emit indices),
      // which the one-batch paths below read from LDS
      if (n > 0) stage_batch<true>(a, c, c.b);
      hits = c.inimg ? a.count[c.pix] : 0;
      load_lists(a, c, s, hits, one_batch, delta);
    } else {
      walk<P, GAUSS>(a, c, s, lam5, delta, evals, steps);
      hits = s.count;
    }
  }
  const int passes = max(1, (wave_max_int(hits) + kChunk - 1) / kChunk);
  if (passes > 1 && lane == 0)
    atomicAdd((unsigned long long*)&a.counters[C_BWD_PASSES], (unsigned long long)(passes - 1));
  float S = 0.f;   // composite of the hits behind the current chunk
  for (int pass = 0; pass < passes; ++pass) {
    const int chunk = passes - 1 - pass;
    if (passes > 1 && !(FUSED && pass == 0)) {
      if (pass > 0) __threadfence_block();   // rows written by other lanes are read back below
      const float T0 = chunk == 0 ? 1.f : chunk == 1 ? s.Tb1 : chunk == 2 ? s.Tb2 : s.Tb3;
      BwdSink r{T0, chunk * kChunk, chunk * kChunk, 1.f, 1.f, 1.f, gD, gN0, gN1, gN2, lam5, a.mode};
      replay(a, c, r, chunk * kChunk, (chunk + 1) * kChunk, hits, one_batch, delta);
    }
    mark(1);
    // back-to-front walk over this chunk
    const int nE = max(0, min(kChunk, hits - chunk * kChunk));
    for (int k = nE - 1; k >= 0; --k) {
      const float T = L.T[k][lane], cv = L.cg[k][lane];
      float omw;
      const float w = splat_weight(L.a[k][lane], lam5, a.mode, omw);
      L.cg[k][lane] = T * (cv - S);
      S = fmaf(w, cv, omw * S);
    }
    // order the chunk by list position (insertion sort, few entries)
    for (int k = 1; k < nE; ++k) {
      const int p = L.pos[k][lane];
      const float T = L.T[k][lane], g = L.cg[k][lane];
      int m = k - 1;
      while (m >= 0 && L.pos[m][lane] > p) {
        L.pos[m + 1][lane] = L.pos[m][lane];
        L.T[m + 1][lane] = L.T[m][lane];
        L.cg[m + 1][lane] = L.cg[m][lane];
        --m;
      }
      L.pos[m + 1][lane] = p;
      L.T[m + 1][lane] = T;
      L.cg[m + 1][lane] = g;
    }
    mark(2);
    // Visit the chunk's candidates in list order, in groups of up to kBatch:
    // gather the next distinct positions (wave minimum of the lanes'
    // cursors); a one-batch list is still staged, longer lists fetch the
    // group's records in parallel; then form the per-pair gradients
    // candidate by candidate.
    int k = 0;
    int npos = nE > 0 ? L.pos[0][lane] : 0x7fffffff;
    while (true) {
      int grp = 0, kk = k, np = npos;
      while (grp < kBatch) {
        const int p = uniform_int(wave_min_int(np));
        if (p == 0x7fffffff) break;
        if (lane == 0) {
          L.gpos[grp] = p;
          if (pass == 0 && !big) L.vis[p >> 5] |= 1u << (p & 31);
        }
        ++grp;
        if (np == p) {
          ++kk;
          np = kk < nE ? L.pos[kk][lane] : 0x7fffffff;
        }
      }
      if (grp == 0) break;
      ncand += grp;
      ++ngrp;
      __syncthreads();
      if (!one_batch) {
        if (lane < grp) {
          const int p = L.gpos[lane];
          const float4* src = reinterpret_cast<const float4*>(&a.recs_s[c.b + p]);
#pragma unroll
          for (int q = 0; q < 7; ++q) stage.head[q][lane] = src[q];
          const float4 tail = src[7];
          stage.pv[lane] = make_float2(tail.z, tail.w);
          stage.em[lane] = a.emit[c.b + p];
        }
        __syncthreads();
      }
      for (int gi = 0; gi < grp; ++gi) {
        const int p = L.gpos[gi];
        const int j = one_batch ? p : gi;   // staging slot of the candidate
        const bool act = npos == p;
        float A[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) A[q] = 0.f;
        if (act) {
          RecHead rec;
          float nrm[3];
          staged(stage, j, rec, nrm);
          const float2 pv = stage.pv[j];
          const float T = L.T[k][lane], gw = L.cg[k][lane];
          const PairGeom g = eval_pair<GAUSS>(rec, c.u, c.v, c.eps, (double)a.z_near, delta);
          const float t = (float)g.t, a32 = (float)g.a;
          const float PX = (float)g.PX, PY = (float)g.PY, den = (float)g.den;
          float omw;
          const float w = splat_weight(a32, lam5, a.mode, omw);
          const float Tw = T * w;
          const bool xp = g.PX > 0.0, yp = g.PY > 0.0;
          float gPX, gPY, grx, gry;   // dL/dP_X, dL/dP_Y, dL/d(radius of the hit's side) along X, Y
          if (GAUSS) {
            // w = exp(-q/2), q = (P_X / s_X)^2 + (P_Y / s_Y)^2
            const float gq = -0.5f * gw * w;
            const float sx = xp ? rec.rxp : rec.rxm, sy = yp ? rec.ryp : rec.rym;
            const float ux = PX / sx, uy = PY / sy;
            gPX = 2.f * gq * ux / sx;
            gPY = 2.f * gq * uy / sy;
            grx = -2.f * gq * ux * ux / sx;
            gry = -2.f * gq * uy * uy / sy;
          } else {
            const float ga = gw * splat_weight_grad(a32, w, omw, lam5, a.mode);
            grx = g.xbranch ? ga : 0.f;
            gry = g.xbranch ? 0.f : ga;
            gPX = xp ? -grx : grx;
            gPY = yp ? -gry : gry;
          }
          // d.vx = (P_X + (p - o).vx) / t, d.vy likewise (x = o + t d)
          const float it = __builtin_amdgcn_rcpf(t);
          const float G = Tw * gD + (gPX * (PX + pv.x) + gPY * (PY + pv.y)) * it;
          const float Gd = G * __builtin_amdgcn_rcpf(den);
          A[0] = gPX;
          A[1] = gPY;
          A[2] = Gd;
          A[3] = gPX * PY - gPY * PX;
          A[4] = Gd * PX;
          A[5] = Gd * PY;
          A[6] = Tw * gN0;
          A[7] = Tw * gN1;
          A[8] = Tw * gN2;
          A[9] = xp ? grx : 0.f;
          A[10] = xp ? 0.f : grx;
          A[11] = yp ? gry : 0.f;
          A[12] = yp ? 0.f : gry;
          ++k;
          npos = k < nE ? L.pos[k][lane] : 0x7fffffff;
        }
        const float tot = wave_sum16(A);
        // lane 4 q holds accumulator q: one store of the row's 13 values
        const int q = lane >> 2;
        if ((lane & 3) == 0 && q < 13) {
          float* row = a.partial + ((size_t)stage.em[j] * a.max_sub + c.sub) * 16;
          if (pass == 0 && !big)
            row[q] = tot;
          else
            row[q] += tot;
        }
      }
      __syncthreads();
    }
    if (pass == 0 && !big) {
      // rows of the list entries this block does not hit
      for (int i = lane; i < n; i += 64)
        if (!((L.vis[i >> 5] >> (i & 31)) & 1u))
          zero_row(a, one_batch ? stage.em[i] : a.emit[c.b + i], c.sub);
    }
    mark(3);
  }
  if (diag && lane == 0) {
    for (int i = 0; i < 4; ++i) dg[D_BWD_SETUP + i] = (long long)ph[i];
    dg[D_BWD_CAND] = (long long)ncand;
    dg[D_BWD_GROUPS] = (long long)ngrp;
    dg[D_BWD_TICKS] = (long long)(ph[0] + ph[1] + ph[2] + ph[3]);
  }
}

template <int P, bool GAUSS, bool PERSIST, bool FUSED>
__global__ __launch_bounds__(64) void render_bwd_kernel(RenderArgs a) {
  if (a.counters[C_OVERFLOW]) return;
  if (!PERSIST) {
    bwd_item<P, GAUSS, FUSED>(a, xcd_item(blockIdx.x, gridDim.x));
    return;
  }
  const int n_groups = (a.n_items + 3) >> 2;
  int stream = blockIdx.x & 7;
  for (int g = claim_group(a.queue, n_groups, stream); g >= 0; g = claim_group(a.queue, n_groups, stream)) {
    for (int item = 4 * g; item < min(4 * g + 4, a.n_items); ++item) {
      bwd_item<P, GAUSS, FUSED>(a, item);
      __syncthreads();
    }
  }
}

// Per plane: sum the partials of each of its records in a fixed order, chain
// the 13 accumulators to the camera-frame center and rotation, map to world
// and to the quaternion, sum over jobs.  One wave per plane.
//   accumulators (sums over pixels and 8x8 blocks; G = dL/dt along the ray):
//     A0 = dL/dP_X, A1 = dL/dP_Y, A2 = G/den, A3 = dP_X P_Y - dP_Y P_X,
//     A4 = (G/den) P_X, A5 = (G/den) P_Y, A6..8 = dL/d(rendered normal),
//     A9..12 = radii (x+, x-, y+, y-)
//   dL/dp = A2 n - A0 vx - A1 vy                          (world frame)
//   dL/domega = A3 n + A5 vx - A4 vy + s n x (R^T A6..8)  (rotation of the frame; s facing sign)
//   dL/dq = 2 (0, dL/domega) (x) q^ / |q|
// The in-plane offsets (P_X, P_Y) enter instead of the hit point, so no sum
// carries the (large) camera distance of the plane.
// Loss sums of job s from the per-8x8-block partials of the forward that
// formed the loss, by 256 threads in the order of the loss calls' own
// reduction (1024 strided partial sums, their wave sums, the 16 wave results
// in order): each thread plays four of those 1024, so the sums have the same
// bits.
__device__ void loss_sums(const RenderArgs& a, int s) {
  __shared__ double lw[16][4];
  const int tid = threadIdx.x, lane = tid & 63;
  const int i0 = a.slots[s].item_begin;
  const int i1 = (s + 1 < a.S) ? a.slots[s + 1].item_begin : a.n_items;
  for (int vw = tid >> 6; vw < 16; vw += 4) {
    double acc[4] = {0, 0, 0, 0};
    for (int i = i0 + vw * 64 + lane; i < i1; i += 1024) {
      const double4 p = *reinterpret_cast<const double4*>(a.loss_in + 4 * (size_t)i);
      acc[0] += p.x; acc[1] += p.y; acc[2] += p.z; acc[3] += p.w;
    }
    for (int q = 0; q < 4; ++q) acc[q] = wave_sum_double(acc[q]);
    if (lane == 0)
      for (int q = 0; q < 4; ++q) lw[vw][q] = acc[q];
  }
  __syncthreads();
  if (tid < 4) {
    double t = lw[0][tid];
    for (int w = 1; w < 16; ++w) t += lw[w][tid];
    a.loss_out[4 * s + tid] = (float)t;
  }
}

// Per plane: the sum of each of its records' partial rows in one fixed order
// whatever the launch shape: the rows in blocks of 64, each block summed
// across a wave (lane l holds row 64 b + l, zeros past the end; wave_sum16),
// the block sums added in block order.  Y = 4: a workgroup per plane, its
// waves sum the blocks w, w + 4, ... of each round of 64 blocks into LDS and
// wave 0 adds them up (few planes: four waves on the rows of a large plane);
// Y = 1: a wave per plane does all of it (many planes: no idle waves).  Same
// bits either way.
template <bool LOSS, int Y, bool ADAM>
__global__ __launch_bounds__(256) void bwd_reduce_kernel(RenderArgs a) {
  __shared__ float part[64][16];   // Y = 4: one round of block sums
  // with LOSS the first n_slots workgroups form the loss sums, one job each
  // (placed last, they cost the 64-room batch's reduction 150 us: measured)
  const int wg = LOSS ? (int)blockIdx.x - a.S : (int)blockIdx.x;
  if (wg < 0) {
    loss_sums(a, wg + a.S);
    return;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  // Y = 4: the dispatcher deals workgroups to the eight XCDs in turn, so the
  // workgroups whose indices agree mod 8 share one XCD's L2; they take a
  // contiguous run of planes, whose parameter, moment and gradient lines are
  // then fetched and written through that L2 alone (a permutation of the
  // planes: each plane's sums are the same)
  int kw = wg;
  if (Y == 4) {
    const int per = a.K >> 3;
    if (wg < 8 * per) kw = (wg & 7) * per + (wg >> 3);
  }
  const int k = Y == 4 ? kw : 4 * wg + w;
  if (k >= a.K) return;
  // the plane's parameters, fetched up front: the chain rule at the end
  // needs them, and their latency hides behind the lookups below
  float pc[3], pq[4];
#pragma unroll
  for (int i = 0; i < 3; ++i) pc[i] = a.center[3 * k + i];
#pragma unroll
  for (int i = 0; i < 4; ++i) pq[i] = a.quat[4 * k + i];
  // ADAM: the update of Sec. 3.3 follows the reduction, lane i < 11 of the
  // wave that writes the gradients taking parameter i (center 0-2, quat 3-6,
  // radii 7-10) with the arithmetic of adam_step_planes (the same moment
  // layout: centers at 3 k, quaternions at 3 K + 4 k, radii at 7 K + 4 k).
  // Its state and bias corrections are fetched and formed here, their
  // latency hidden by the reduction.  Plane k's parameters and moments are
  // read and written by plane k's reduction only.
  const int ugrp = lane < 3 ? 0 : lane < 7 ? 1 : 2;
  const int upi = ugrp == 0 ? 3 * k + lane : 4 * k + lane - (ugrp == 1 ? 3 : 7);
  const int umj = upi + (ugrp == 0 ? 0 : ugrp == 1 ? 3 * a.K : 7 * a.K);
  float* const up = ugrp == 0 ? a.upd_p[0] : ugrp == 1 ? a.upd_p[1] : a.upd_p[2];
  const bool uown = ADAM && lane < 11 && (Y == 1 || w == 0);
  float um = 0.f, uv = 0.f, upar = 0.f;
  double bc1 = 1.0, bc2 = 1.0;
  if (uown) {
    um = a.upd_m[umj];
    uv = a.upd_v[umj];
    upar = up[upi];
    adam_bias(a.upd_b1, a.upd_b2, a.upd_step[0], bc1, bc2);
  }
  double gp[3] = {0, 0, 0}, gw[3] = {0, 0, 0}, gr[4] = {0, 0, 0, 0};
  double qn[4] = {0, 0, 0, 0}, qnorm = 0;
  const bool ok = !a.counters[C_OVERFLOW];
  // the slots holding plane k, in slot order, 64 slots per lookup (one slot
  // per lane, whose fields the wave then reads from that lane); with sorted
  // plane ranges they are a run starting at the first slot whose range ends
  // after k.  (With Y = 4 every wave of the workgroup finds the same slots.)
  int s0 = 0;
  if (a.slots_sorted && a.S > 64) {
    int lo = 0, hi = a.S;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (a.slots[mid].plane_end > k) hi = mid; else lo = mid + 1;
    }
    s0 = lo;
  }
  for (int sb = s0; sb < a.S && ok; sb += 64) {
    const int sl_i = sb + lane;
    bool in = false, past = false;
    int f_pb = 0, f_cam = 0, f_rb = 0, f_nsub = 0;
    if (sl_i < a.S) {
      const ps_slot& q = a.slots[sl_i];
      f_pb = q.plane_begin;
      f_cam = q.cam;
      f_rb = q.rec_begin;
      f_nsub = (q.tile_w >> 3) * (q.tile_h >> 3);
      in = k >= f_pb && k < q.plane_end && f_cam >= 0 && f_cam < a.n_cams;
      past = f_pb > k;
    }
    uint64_t m = ballot(in);
    const bool stop = a.slots_sorted && ballot(past) != 0;
    while (m) {
      const int j = __ffsll((unsigned long long)m) - 1;
      m &= m - 1;
      const int cam_i = __builtin_amdgcn_readlane(f_cam, j);
      const int r = __builtin_amdgcn_readlane(f_rb, j) + (k - __builtin_amdgcn_readlane(f_pb, j));
      const int nsub = __builtin_amdgcn_readlane(f_nsub, j);
      const ps_camera cam = a.cams[cam_i];
      if (a.recs[r].cull) continue;
      const int rows = a.rec_cnt[r] * nsub;
      const int e0 = a.rec_off[r] + a.rbase[r / kScanChunk];
      // row i of the record: partial row (e0 + i / nsub, i % nsub)
      auto row_of = [&](int i, float (&v)[16]) {
        if (i < rows) {
          const int e = e0 + i / nsub, sbk = i % nsub;
          const float* rowp = a.partial + ((size_t)e * a.max_sub + sbk) * 16;
          const float4* row = (const float4*)rowp;
          const float4 r0 = row[0], r1 = row[1], r2 = row[2];
          v[0] = r0.x; v[1] = r0.y; v[2] = r0.z; v[3] = r0.w;
          v[4] = r1.x; v[5] = r1.y; v[6] = r1.z; v[7] = r1.w;
          v[8] = r2.x; v[9] = r2.y; v[10] = r2.z; v[11] = r2.w;
          v[12] = rowp[12];
        } else {
#pragma unroll
          for (int q = 0; q < 13; ++q) v[q] = 0.f;
        }
        v[13] = v[14] = v[15] = 0.f;
      };
      const int nblk = (rows + 63) >> 6;
      float acc = 0.f;   // lane 4 q + r: the sum of accumulator q so far
      if (Y == 1) {
        for (int b = 0; b < nblk; b += 2) {   // two blocks in flight
          float v0[16], v1[16];
          row_of(64 * b + lane, v0);
          row_of(64 * (b + 1) + lane, v1);
          acc += wave_sum16(v0);
          if (b + 1 < nblk) acc += wave_sum16(v1);
        }
      } else {
        for (int r0 = 0; r0 < nblk; r0 += 64) {
          const int nb = min(64, nblk - r0);
          for (int b = w; b < nb; b += 8) {   // blocks b and b + 4 in flight
            float v[2][16];
#pragma unroll
            for (int u = 0; u < 2; ++u) row_of(64 * (r0 + b + 4 * u) + lane, v[u]);
#pragma unroll
            for (int u = 0; u < 2; ++u)
              if (b + 4 * u < nb) {
                const float t = wave_sum16(v[u]);
                if ((lane & 3) == 0) part[b + 4 * u][lane >> 2] = t;
              }
          }
          __syncthreads();
          if (w == 0)
            for (int b = 0; b < nb; ++b) acc += part[b][lane >> 2];
          __syncthreads();
        }
      }
      float S[13];
#pragma unroll
      for (int q = 0; q < 13; ++q) S[q] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(acc), 4 * q));
      Frame f;
      if (!plane_frame(pc, pq, 0, cam, f)) continue;
      for (int q = 0; q < 4; ++q) qn[q] = f.q[q];
      qnorm = f.qnorm;
      const double sg = a.two_sided ? (f.h > 0.0 ? -1.0 : 1.0) : 1.0;
      double gs[3];   // s R^T dL/d(rendered normal)
      for (int i = 0; i < 3; ++i)
        gs[i] = sg * ((double)cam.R[i] * S[6] + (double)cam.R[3 + i] * S[7] + (double)cam.R[6 + i] * S[8]);
      const double nxg[3] = {f.n[1] * gs[2] - f.n[2] * gs[1], f.n[2] * gs[0] - f.n[0] * gs[2],
                             f.n[0] * gs[1] - f.n[1] * gs[0]};
      for (int i = 0; i < 3; ++i) {
        gp[i] += (double)S[2] * f.n[i] - (double)S[0] * f.vx[i] - (double)S[1] * f.vy[i];
        gw[i] += (double)S[3] * f.n[i] + (double)S[5] * f.vx[i] - (double)S[4] * f.vy[i] + nxg[i];
      }
      for (int q = 0; q < 4; ++q) gr[q] += S[9 + q];
    }
    if (stop) break;
  }
  if (Y == 1 || w == 0) {
    // gp, gw, gr, qn and qnorm are the same in every lane of the wave
    float gc[3], grf[4], gq[4] = {0.f, 0.f, 0.f, 0.f};
    for (int i = 0; i < 3; ++i) gc[i] = (float)gp[i];
    for (int q = 0; q < 4; ++q) grf[q] = (float)gr[q];
    // 2 (0, w) (x) q^  =  2 (-(w . v), q0 w + w x v),  v = (q1, q2, q3)
    if (qnorm > 0) {
      const double s2 = 2.0 / qnorm;
      const double v0 = qn[1], v1 = qn[2], v2 = qn[3];
      gq[0] = (float)(s2 * -(gw[0] * v0 + gw[1] * v1 + gw[2] * v2));
      gq[1] = (float)(s2 * (qn[0] * gw[0] + (gw[1] * v2 - gw[2] * v1)));
      gq[2] = (float)(s2 * (qn[0] * gw[1] + (gw[2] * v0 - gw[0] * v2)));
      gq[3] = (float)(s2 * (qn[0] * gw[2] + (gw[0] * v1 - gw[1] * v0)));
    }
    if (lane == 0) {
      for (int i = 0; i < 3; ++i) a.g_center[3 * k + i] = gc[i];
      for (int q = 0; q < 4; ++q) a.g_radii[4 * k + q] = grf[q];
      for (int q = 0; q < 4; ++q) a.g_quat[4 * k + q] = gq[q];
    }
    if (uown) {
      float g = gc[0];
      g = lane == 1 ? gc[1] : g;
      g = lane == 2 ? gc[2] : g;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        g = lane == 3 + q ? gq[q] : g;
        g = lane == 7 + q ? grf[q] : g;
      }
      const float lr = ugrp == 0 ? a.upd_lr[0] : ugrp == 1 ? a.upd_lr[1] : a.upd_lr[2];
      const float x = adam_apply(upar, g, um, uv, lr, a.upd_b1, a.upd_b2, a.upd_eps, bc1, bc2);
      a.upd_m[umj] = um;
      a.upd_v[umj] = uv;
      up[upi] = ugrp == 2 ? fmaxf(x, a.upd_rmin) : x;
    }
  }
}

// Pending-hit buffer size: ps_params.flags bits 4-5 select 6 (default), 4, 8 or 12.
// A larger buffer sends fewer pixels to the round-based continuation at the
// cost of registers (occupancy); the autotuner picks it with the tile shape.
inline int pending_of(int flags) {
  switch ((flags >> 4) & 3) {
    case 1: return 4;
    case 2: return 8;
    case 3: return 12;
    default: return 6;
  }
}

int fill_args(const ps_layout* L, void* ws, const ps_camera* cams, int n_cams, const float* lambda,
              const ps_params* prm, RenderArgs& a, const char* who) {
  int rc = ps_check_ws(L, ws, who);
  if (rc) return rc;
  if (!cams || !lambda || !prm) return ps_set_error(PS_ERR_INVALID, "%s: null pointer", who);
  if (n_cams <= 0) return ps_set_error(PS_ERR_INVALID, "%s: n_cams <= 0", who);
  if (!(prm->tau > 0.f && prm->tau < 1.f) || !(prm->z_near > 0.f) || prm->M < 1 || prm->M > kMaxM ||
      (prm->weight_mode < 0 || prm->weight_mode > 2))
    return ps_set_error(PS_ERR_INVALID, "%s: bad ps_params", who);
  char* base = (char*)ws;
  memset(&a, 0, sizeof(a));
  a.slots = (const ps_slot*)(base + L->region[R_SLOTS]);
  a.S = L->n_slots;
  a.slots_sorted = L->slots_sorted;
  a.n_items = L->n_items;
  a.recs = (const Rec*)(base + L->region[R_REC]);
  a.items = (const ItemDesc*)(base + L->region[R_ITEMS]);
  a.recs_s = (const Rec*)(base + L->region[R_RECS_S]);
  a.keys = (const uint64_t*)(base + L->region[R_KEYS_S]);
  a.emit = (const uint32_t*)(base + L->region[R_EMIT_S]);
  a.rec_cnt = (const int*)(base + L->region[R_REC_CNT]);
  a.rec_off = (const int*)(base + L->region[R_REC_OFF]);
  a.rbase = (const int*)(base + L->region[R_SCAN]) + scan_chunks(L->n_tiles, L->n_records);
  a.cams = cams;
  a.n_cams = n_cams;
  a.lambda = lambda;
  a.tau = prm->tau; a.z_near = prm->z_near; a.M = prm->M; a.mode = prm->weight_mode;
  a.flog = filter_log((double)prm->tau, prm->weight_mode);
  a.flags = prm->flags; a.two_sided = prm->two_sided;
  a.counters = (long long*)(base + L->region[R_COUNTERS]);
  a.diag = (long long*)(base + L->region[R_DIAG]);
  a.partial = (float*)(base + L->region[R_PARTIAL]);
  a.max_sub = L->max_sub;
  a.queue = (unsigned long long*)(base + L->region[R_QUEUE]);
  return PS_OK;
}

}  // namespace

// Workgroups of a render kernel resident on the device at once (cached per
// kernel and device).  A launch with more 8x8 items than that runs
// persistent: the grid is this many workgroups and they claim items from
// the work queue; a smaller launch keeps one workgroup per item (no claim).
static int resident_grid(const void* kernel, hipStream_t st, int* out) {
  struct Entry { const void* k; int dev; int n; };
  static Entry cache[64];
  static int n_cache = 0;
  static std::mutex mu;
  int dev = 0;
  if (st) {
    hipDevice_t d;
    PS_HIP_CHECK(hipStreamGetDevice(st, &d));
    dev = (int)d;
  } else {
    PS_HIP_CHECK(hipGetDevice(&dev));
  }
  std::lock_guard<std::mutex> lock(mu);
  for (int i = 0; i < n_cache; ++i)
    if (cache[i].k == kernel && cache[i].dev == dev) {
      *out = cache[i].n;
      return PS_OK;
    }
  int per_cu = 0, cus = 0;
  PS_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 64, 0));
  PS_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int n = per_cu > 0 && cus > 0 ? per_cu * cus : 1;
  if (n_cache < 64) cache[n_cache++] = Entry{kernel, dev, n};
  *out = n;
  return PS_OK;
}

// One workgroup per item, or persistent when the items are more than four
// times what the GPU holds resident at once (ps_params.flags bit 8 keeps one
// workgroup per item).  The forward is persistent only with flags bit 9: its
// persistent form needs 150 VGPRs against 123 (three waves per SIMD instead
// of four), and on the 64-room batch it took 1.02 ms against 0.70 ms one
// workgroup per item; the backward (LDS-bound at eight workgroups per
// compute unit either way) gains 3 % from it.
template <class K1, class KP>
static int launch_items(K1 k1, KP kp, RenderArgs& a, unsigned long long* queue, bool persist_ok, hipStream_t st) {
  int cap1 = 0, cap = 0;
  int rc = resident_grid(reinterpret_cast<const void*>(k1), st, &cap1);
  if (rc) return rc;
  rc = resident_grid(reinterpret_cast<const void*>(kp), st, &cap);
  if (rc) return rc;
  if (!persist_ok || a.n_items <= 4 * cap1 || (a.flags & kFlagNoPersist)) {
    a.queue = nullptr;
    hipLaunchKernelGGL(k1, dim3(a.n_items), dim3(64), 0, st, a);
    return PS_OK;
  }
  a.queue = queue;
  hipLaunchKernelGGL(kp, dim3(cap), dim3(64), 0, st, a);
  hipLaunchKernelGGL(queue_reset_kernel, dim3(1), dim3(64), 0, st, queue);
  return PS_OK;
}

template <bool GAUSS>
static int launch_fwd_g(RenderArgs& a, hipStream_t st) {
  unsigned long long* q = a.queue;
  const bool pp = a.flags & kFlagPersistFwd;
  switch (pending_of(a.flags)) {
    case 4: return launch_items(render_fwd_kernel<4, GAUSS, false>, render_fwd_kernel<4, GAUSS, true>, a, q, pp, st);
    case 8: return launch_items(render_fwd_kernel<8, GAUSS, false>, render_fwd_kernel<8, GAUSS, true>, a, q, pp, st);
    case 12:
      return launch_items(render_fwd_kernel<12, GAUSS, false>, render_fwd_kernel<12, GAUSS, true>, a, q, pp, st);
    default: return launch_items(render_fwd_kernel<6, GAUSS, false>, render_fwd_kernel<6, GAUSS, true>, a, q, pp, st);
  }
}
template <bool GAUSS, bool FUSED>
static int launch_bwd_g(RenderArgs& a, hipStream_t st) {
  unsigned long long* q = a.queue + 8 * kQueueStride;
  switch (pending_of(a.flags)) {
    case 4:
      return launch_items(render_bwd_kernel<4, GAUSS, false, FUSED>, render_bwd_kernel<4, GAUSS, true, FUSED>, a, q,
                          true, st);
    case 8:
      return launch_items(render_bwd_kernel<8, GAUSS, false, FUSED>, render_bwd_kernel<8, GAUSS, true, FUSED>, a, q,
                          true, st);
    case 12:
      return launch_items(render_bwd_kernel<12, GAUSS, false, FUSED>, render_bwd_kernel<12, GAUSS, true, FUSED>, a, q,
                          true, st);
    default:
      return launch_items(render_bwd_kernel<6, GAUSS, false, FUSED>, render_bwd_kernel<6, GAUSS, true, FUSED>, a, q,
                          true, st);
  }
}

// The Gaussian weight (mode 2) has kernels of its own, so the other modes
// carry no per-candidate test of the mode.
static int launch_fwd(RenderArgs& a, void* stream) {
  if (a.n_items == 0) return PS_OK;
  const int rc = a.mode == 2 ? launch_fwd_g<true>(a, (hipStream_t)stream) : launch_fwd_g<false>(a, (hipStream_t)stream);
  if (rc) return rc;
  PS_HIP_CHECK(hipGetLastError());
  return PS_OK;
}
// fused: the fitting step's forward, loss and backward in one launch (the
// forward-with-loss fields of `a` set as well)
template <bool LOSS, bool ADAM>
static void launch_reduce(const RenderArgs& a, int nwg, bool per_wave, hipStream_t st) {
  const dim3 grid(nwg + (LOSS ? a.S : 0));
  if (per_wave)
    hipLaunchKernelGGL((bwd_reduce_kernel<LOSS, 1, ADAM>), grid, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((bwd_reduce_kernel<LOSS, 4, ADAM>), grid, dim3(256), 0, st, a);
}

static int launch_bwd(RenderArgs& a, int K, void* stream, bool fused = false) {
  hipStream_t st = (hipStream_t)stream;
  if (a.n_items > 0) {
    int rc;
    if (fused)
      rc = a.mode == 2 ? launch_bwd_g<true, true>(a, st) : launch_bwd_g<false, true>(a, st);
    else
      rc = a.mode == 2 ? launch_bwd_g<true, false>(a, st) : launch_bwd_g<false, false>(a, st);
    if (rc) return rc;
  }
  // a wave per plane for many planes, a workgroup per plane for few (the
  // same bits either way); ps_params.flags bit 10 asks for a wave per plane
  const bool per_wave = K >= kReduceWaveMin || (a.flags & kFlagReduceWave);
  const int nwg = per_wave ? (K + 3) / 4 : K;
  // with the Adam state set the planes are updated: by the reduction when it
  // has a workgroup per plane (one launch fewer per step), by a kernel of its
  // own after a wave-per-plane reduction (many planes: there the update's
  // latency, two float64 powers and the parameter reads, would lengthen
  // every round of waves).  The bits are the same either way.
  const bool adam = a.upd_m && K > 0, fold = adam && !per_wave;
  if (a.loss_out) {
    if (fold) launch_reduce<true, true>(a, nwg, per_wave, st);
    else launch_reduce<true, false>(a, nwg, per_wave, st);
  } else if (K > 0) {
    if (fold) launch_reduce<false, true>(a, nwg, per_wave, st);
    else launch_reduce<false, false>(a, nwg, per_wave, st);
  }
  PS_HIP_CHECK(hipGetLastError());
  if (adam && !fold)
    return adam_step_planes(a.upd_p[0], a.upd_p[1], a.upd_p[2], a.g_center, a.g_quat, a.g_radii, a.upd_m, a.upd_v, K,
                            a.upd_step, a.upd_lr[0], a.upd_lr[1], a.upd_lr[2], a.upd_b1, a.upd_b2, a.upd_eps,
                            a.upd_rmin, stream);
  return PS_OK;
}

static int bwd_args(const ps_layout* L, void* ws, const float* center, const float* quat, const float* radii, int K,
                    const ps_camera* cams, int n_cams, const float* lambda, const ps_params* prm,
                    const float* g_depth, const float* g_normal, float* g_center, float* g_quat, float* g_radii,
                    RenderArgs& a, const char* who, bool upstream = true) {
  int rc = fill_args(L, ws, cams, n_cams, lambda, prm, a, who);
  if (rc) return rc;
  // an empty plane set (K = 0) may come with null plane and gradient arrays;
  // upstream false: the loss gradient is formed inside (plane_render_step)
  if ((upstream && (!g_depth || !g_normal)) || K < 0 ||
      (K > 0 && (!center || !quat || !radii || !g_center || !g_quat || !g_radii)))
    return ps_set_error(PS_ERR_INVALID, "%s: null pointer or K < 0", who);
  if (K < L->n_planes) return ps_set_error(PS_ERR_INVALID, "%s: K=%d < planes referenced %d", who, K, L->n_planes);
  a.g_depth = g_depth; a.g_normal = g_normal;
  a.center = center; a.quat = quat; a.K = K;
  a.g_center = g_center; a.g_quat = g_quat; a.g_radii = g_radii;
  return PS_OK;
}

extern "C" int plane_render_fwd(const ps_layout* L, void* ws, const ps_camera* cams, int n_cams,
                                const float* lambda, const ps_params* prm, float* depth, float* normal,
                                float* trans, int32_t* count, void* stream) {
  RenderArgs a;
  int rc = fill_args(L, ws, cams, n_cams, lambda, prm, a, "plane_render_fwd");
  if (rc) return rc;
  if (!depth || !normal) return ps_set_error(PS_ERR_INVALID, "plane_render_fwd: null output");
  a.depth = depth;
  a.normal = normal;
  a.trans = trans;
  a.count = count;
  return launch_fwd(a, stream);
}

extern "C" int plane_render_fwd_loss(const ps_layout* L, void* ws, const ps_camera* cams, int n_cams,
                                     const float* lambda, const ps_params* prm, float* depth, float* normal,
                                     const float* tgt_depth, const float* tgt_normal, const uint8_t* mask,
                                     const int64_t* tgt_off, int n_tgt, float a_cos, float a_nl1, float a_d,
                                     float* loss, float* g_depth, float* g_normal, void* stream) {
  RenderArgs a;
  int rc = fill_args(L, ws, cams, n_cams, lambda, prm, a, "plane_render_fwd_loss");
  if (rc) return rc;
  if (!depth || !normal || !tgt_depth || !tgt_normal || !g_depth || !g_normal || (tgt_off && n_tgt <= 0))
    return ps_set_error(PS_ERR_INVALID, "plane_render_fwd_loss: bad argument");
  a.depth = depth;
  a.normal = normal;
  a.loss.Dt = tgt_depth; a.loss.Nt = tgt_normal; a.loss.mask = mask;
  a.loss.tgt_off = tgt_off; a.loss.n_cams = tgt_off ? n_tgt : 0;
  a.loss.a_cos = a_cos; a.loss.a_nl1 = a_nl1; a.loss.a_d = a_d;
  a.loss.gD = g_depth; a.loss.gN = g_normal;
  a.loss_part = (double*)((char*)ws + L->region[R_LOSS]);
  rc = launch_fwd(a, stream);
  if (rc) return rc;
  // without loss the per-block partials stay for plane_render_bwd_adam
  return loss ? ps_loss_reduce(L, ws, loss, stream) : PS_OK;
}

extern "C" int plane_render_bwd(const ps_layout* L, void* ws, const float* center, const float* quat,
                                const float* radii, int K, const ps_camera* cams, int n_cams,
                                const float* lambda, const ps_params* prm, const float* g_depth,
                                const float* g_normal, float* g_center, float* g_quat, float* g_radii,
                                void* stream) {
  RenderArgs a;
  int rc = bwd_args(L, ws, center, quat, radii, K, cams, n_cams, lambda, prm, g_depth, g_normal, g_center, g_quat,
                    g_radii, a, "plane_render_bwd");
  if (rc) return rc;
  return launch_bwd(a, K, stream);
}

// The Adam state of the reduction's update (null m when K = 0: no update).
static void set_adam(RenderArgs& a, float* center, float* quat, float* radii, float* m, float* v,
                     const int32_t* step, float lr_center, float lr_quat, float lr_radii, float beta1, float beta2,
                     float eps, float r_min) {
  a.upd_p[0] = center; a.upd_p[1] = quat; a.upd_p[2] = radii;
  a.upd_m = m; a.upd_v = v; a.upd_step = step;
  a.upd_lr[0] = lr_center; a.upd_lr[1] = lr_quat; a.upd_lr[2] = lr_radii;
  a.upd_b1 = beta1; a.upd_b2 = beta2; a.upd_eps = eps; a.upd_rmin = r_min;
}

extern "C" int plane_render_bwd_adam(const ps_layout* L, void* ws, float* center, float* quat, float* radii, int K,
                                     const ps_camera* cams, int n_cams, const float* lambda, const ps_params* prm,
                                     const float* g_depth, const float* g_normal, float* g_center, float* g_quat,
                                     float* g_radii, float* m, float* v, const int32_t* step, float lr_center,
                                     float lr_quat, float lr_radii, float beta1, float beta2, float eps, float r_min,
                                     float* loss, void* stream) {
  RenderArgs a;
  int rc = bwd_args(L, ws, center, quat, radii, K, cams, n_cams, lambda, prm, g_depth, g_normal, g_center, g_quat,
                    g_radii, a, "plane_render_bwd_adam");
  if (rc) return rc;
  if (K > 0 && (!m || !v || !step)) return ps_set_error(PS_ERR_INVALID, "plane_render_bwd_adam: null Adam state");
  if (!(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return ps_set_error(PS_ERR_INVALID, "plane_render_bwd_adam: bad beta / eps");
  if (loss) {
    a.loss_out = loss;
    a.loss_in = (const double*)((char*)ws + L->region[R_LOSS]);
  }
  set_adam(a, center, quat, radii, m, v, step, lr_center, lr_quat, lr_radii, beta1, beta2, eps, r_min);
  return launch_bwd(a, K, stream);
}

extern "C" int plane_render_step(const ps_layout* L, void* ws, float* center, float* quat, float* radii, int K,
                                 const ps_camera* cams, int n_cams, const float* lambda, const ps_params* prm,
                                 float* depth, float* normal, const float* tgt_depth, const float* tgt_normal,
                                 const uint8_t* mask, const int64_t* tgt_off, int n_tgt, float a_cos, float a_nl1,
                                 float a_d, float* g_depth, float* g_normal, float* g_center, float* g_quat,
                                 float* g_radii, float* m, float* v, const int32_t* step, float lr_center,
                                 float lr_quat, float lr_radii, float beta1, float beta2, float eps, float r_min,
                                 float* loss, void* stream) {
  RenderArgs a;
  int rc = bwd_args(L, ws, center, quat, radii, K, cams, n_cams, lambda, prm, g_depth, g_normal, g_center, g_quat,
                    g_radii, a, "plane_render_step", false);
  if (rc) return rc;
  if (!tgt_depth || !tgt_normal || (tgt_off && n_tgt <= 0) || !depth != !normal || !g_depth != !g_normal)
    return ps_set_error(PS_ERR_INVALID, "plane_render_step: bad argument");
  if (K > 0 && (!m || !v || !step)) return ps_set_error(PS_ERR_INVALID, "plane_render_step: null Adam state");
  if (!(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return ps_set_error(PS_ERR_INVALID, "plane_render_step: bad beta / eps");
  if (a.flags & kFlagDiag)
    return ps_set_error(PS_ERR_INVALID, "plane_render_step: the walk statistics (flags bit 6) are the separate "
                                        "calls'");
  a.depth = depth;
  a.normal = normal;
  a.loss.Dt = tgt_depth; a.loss.Nt = tgt_normal; a.loss.mask = mask;
  a.loss.tgt_off = tgt_off; a.loss.n_cams = tgt_off ? n_tgt : 0;
  a.loss.a_cos = a_cos; a.loss.a_nl1 = a_nl1; a.loss.a_d = a_d;
  a.loss.gD = g_depth; a.loss.gN = g_normal;
  a.loss_part = (double*)((char*)ws + L->region[R_LOSS]);
  if (loss) {
    a.loss_out = loss;
    a.loss_in = a.loss_part;
  }
  set_adam(a, center, quat, radii, m, v, step, lr_center, lr_quat, lr_radii, beta1, beta2, eps, r_min);
  return launch_bwd(a, K, stream, true);
}

extern "C" int plane_render_fwd_lists(const ps_layout* L, void* ws, const ps_camera* cams, int n_cams,
                                      const float* lambda, const ps_params* prm, float* depth, float* normal,
                                      int32_t* list_pos, float* list_a, float* list_T, int32_t* list_count,
                                      void* stream) {
  RenderArgs a;
  int rc = fill_args(L, ws, cams, n_cams, lambda, prm, a, "plane_render_fwd_lists");
  if (rc) return rc;
  if (!depth || !normal || !list_pos || !list_a || !list_T || !list_count)
    return ps_set_error(PS_ERR_INVALID, "plane_render_fwd_lists: null pointer");
  a.depth = depth;
  a.normal = normal;
  a.count = list_count;
  a.lst_pos = list_pos; a.lst_a = list_a; a.lst_T = list_T;
  a.lst_stride = L->n_pixels;
  return launch_fwd(a, stream);
}

extern "C" int plane_render_bwd_lists(const ps_layout* L, void* ws, const float* center, const float* quat,
                                      const float* radii, int K, const ps_camera* cams, int n_cams,
                                      const float* lambda, const ps_params* prm, const float* g_depth,
                                      const float* g_normal, const int32_t* list_pos, const float* list_a,
                                      const int32_t* list_count, float* g_center, float* g_quat, float* g_radii,
                                      void* stream) {
  RenderArgs a;
  int rc = bwd_args(L, ws, center, quat, radii, K, cams, n_cams, lambda, prm, g_depth, g_normal, g_center, g_quat,
                    g_radii, a, "plane_render_bwd_lists");
  if (rc) return rc;
  if (!list_pos || !list_a || !list_count) return ps_set_error(PS_ERR_INVALID, "plane_render_bwd_lists: null list");
  a.lst_pos = const_cast<int32_t*>(list_pos);
  a.lst_a = const_cast<float*>(list_a);
  a.count = const_cast<int32_t*>(list_count);
  a.lst_stride = L->n_pixels;
  return launch_bwd(a, K, stream);
}
