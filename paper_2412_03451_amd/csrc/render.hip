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

#include "ps_internal.h"

using namespace ps;

int ps_check_ws(const ps_layout* L, const void* ws, const char* who);

namespace {

struct RenderArgs {
  const ps_slot* slots;
  int S, n_items;
  const Rec* recs;
  const int* tile_off;
  const uint64_t* keys;
  const uint32_t* emit;
  const int* rec_cnt;
  const int* rec_off;
  const ps_camera* cams;
  int n_cams;
  const float* lambda;
  float tau, z_near;
  int M, mode, flags, two_sided;
  long long* counters;
  float* depth;
  float* normal;
  float* trans;      // optional: final transmittance per pixel
  int32_t* count;    // optional: committed hits per pixel
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
};

struct ItemCtx {
  int slot;
  int b, e;          // list range in keys[]
  int sub;           // 8x8 block index inside the tile
  int px, py;        // this lane's pixel
  bool inimg;
  int bx0, bx1, by0, by1;  // pixel box of the block (clipped to the image)
  double u, v, eps;  // pixel center, |den| threshold
  float du, dv;      // camera-frame ray (du, dv, 1)
  int64_t pix;       // index of the pixel in the depth array
  int64_t pix_off, HW;
  ps_camera cam;
};

// 0: block inside the image; 1: block entirely outside (partial tile); 2: bad camera
__device__ inline int item_setup(const RenderArgs& a, int item, ItemCtx& c) {
  const int s = find_slot_by_item(a.slots, a.S, item);
  const ps_slot sl = a.slots[s];
  if (sl.cam < 0 || sl.cam >= a.n_cams) return 2;
  c.slot = s;
  const int local = item - sl.item_begin;
  const int sub_w = sl.tile_w >> 3;
  const int sub_per = sub_w * (sl.tile_h >> 3);
  const int tile = local / sub_per;
  c.sub = local - tile * sub_per;
  const int tx = tile % sl.tiles_x, ty = tile / sl.tiles_x;
  const int ox = tx * sl.tile_w + (c.sub % sub_w) * 8;
  const int oy = ty * sl.tile_h + (c.sub / sub_w) * 8;
  const int gt = sl.tile_begin + tile;
  c.b = a.tile_off[gt];
  c.e = a.tile_off[gt + 1];
  const int lane = threadIdx.x;
  c.px = ox + (lane & 7);
  c.py = oy + (lane >> 3);
  c.inimg = c.px < sl.width && c.py < sl.height;
  c.bx0 = ox; c.bx1 = min(ox + 7, sl.width - 1);
  c.by0 = oy; c.by1 = min(oy + 7, sl.height - 1);
  c.cam = a.cams[sl.cam];
  c.u = c.px + 0.5;
  c.v = c.py + 0.5;
  const double du = (c.u - (double)c.cam.cx) / (double)c.cam.fx;
  const double dv = (c.v - (double)c.cam.cy) / (double)c.cam.fy;
  c.du = (float)du;
  c.dv = (float)dv;
  c.eps = 1e-12 * sqrt(du * du + dv * dv + 1.0);
  c.pix_off = sl.pix_off;
  c.HW = (int64_t)sl.width * sl.height;
  c.pix = sl.pix_off + (int64_t)c.py * sl.width + c.px;
  return (ox < sl.width && oy < sl.height) ? 0 : 1;
}

// Sorted buffer of pending hits (ascending (t, record)), in registers.  Each
// entry keeps the float32 a* of the hit; weights are formed at commit time.
template <int P>
struct Pending {
  float t[P];
  int r[P];
  float a[P];
  int pos[P];
  int n;
  float ot; int orr;   // key of the opaque pending hit, +inf if none
  float tt; int tr;    // key of the last pending hit

  __device__ void reset() {
    n = 0;
    ot = INFINITY; orr = 0x7fffffff;
    tt = -INFINITY; tr = -1;
  }

  // false: the buffer is full and the hit may still be among the first M
  __device__ bool insert(float nt, int nr, float na, bool opq, int npos, int committed, int M) {
    if (key_less(ot, orr, nt, nr)) return true;              // behind an opaque hit
    const bool fullm = committed + n >= M;
    if (fullm && (n == 0 || !key_less(nt, nr, tt, tr))) return true;  // beyond the first M
    if (!fullm && n == P) return false;
    if (fullm) {                                             // the old last entry leaves the first M
      n -= 1;
      ot = INFINITY; orr = 0x7fffffff;                       // an opaque hit is always the last entry
    }
    int at = 0;
#pragma unroll
    for (int k = 0; k < P; ++k)
      if (k < n && key_less(t[k], r[k], nt, nr)) ++at;
#pragma unroll
    for (int k = P - 1; k >= 1; --k)
      if (k > at && k <= n) {
        t[k] = t[k - 1]; r[k] = r[k - 1]; a[k] = a[k - 1]; pos[k] = pos[k - 1];
      }
#pragma unroll
    for (int k = 0; k < P; ++k)
      if (k == at) { t[k] = nt; r[k] = nr; a[k] = na; pos[k] = npos; }
    n += 1;
    if (opq) {   // everything behind an opaque hit is hidden
      n = at + 1;
      ot = nt; orr = nr;
    }
#pragma unroll
    for (int k = 0; k < P; ++k)
      if (k == n - 1) { tt = t[k]; tr = r[k]; }
    return true;
  }

  __device__ void pop(float& ft, int& fr, float& fa, int& fpos) {
    ft = t[0]; fr = r[0]; fa = a[0]; fpos = pos[0];
#pragma unroll
    for (int k = 0; k + 1 < P; ++k) { t[k] = t[k + 1]; r[k] = r[k + 1]; a[k] = a[k + 1]; pos[k] = pos[k + 1]; }
    n -= 1;
    if (n == 0) { tt = -INFINITY; tr = -1; ot = INFINITY; orr = 0x7fffffff; }
  }
};

// Walk the tile list of one 8x8 block and hand every committed hit, in exact
// per-ray order, to sink.commit(t, record, a*, list position).
template <int P, class Sink>
__device__ void walk(const RenderArgs& a, const ItemCtx& c, Sink& sink, float lam5, double delta) {
  Pending<P> pd;
  pd.reset();
  bool slow = (a.flags & 1) && c.inimg;
  bool done = !c.inimg || slow || sink.finished(a.M);
  float lt = -INFINITY;
  int lr = -1;
  for (int i = c.b; i < c.e; ++i) {
    if (ballot(!done) == 0) break;
    const uint64_t key = a.keys[i];
    const int ri = (int)(uint32_t)key;
    const float tlb_next = (i + 1 < c.e) ? __uint_as_float((uint32_t)(a.keys[i + 1] >> 32)) : INFINITY;
    const Rec& rec = a.recs[ri];
    const bool overlap = !(rec.px1 < c.bx0 || rec.px0 > c.bx1 || rec.py1 < c.by0 || rec.py0 > c.by1);
    if (overlap) {
      const PairGeom g = eval_pair(rec, c.u, c.v, c.eps, (double)a.z_near, delta);
      const bool hit = g.ok && !done;
      if (ballot(hit)) {
        if (hit) {
          const float t32 = (float)g.t;
          const float a32 = (float)g.a;
          if (!pd.insert(t32, ri, a32, a.mode == 0 && a32 >= 0.f, i - c.b, sink.count, a.M)) {
            slow = true;
            done = true;
          }
        }
      }
    }
    bool want = !done && pd.n > 0 && pd.t[0] < tlb_next;
    if (ballot(want)) {
      while (want) {
        float ft, fa; int fr, fp;
        pd.pop(ft, fr, fa, fp);
        sink.commit(a, c, ft, fr, fa, fp);
        lt = ft; lr = fr;
        if (sink.finished(a.M)) { done = true; break; }
        want = pd.n > 0 && pd.t[0] < tlb_next;
      }
    }
  }
  const uint64_t slow_mask = ballot(slow);
  if (slow_mask && threadIdx.x == 0)
    atomicAdd((unsigned long long*)&a.counters[C_SLOW], (unsigned long long)__popcll(slow_mask));
  if (slow) {
    // exact fallback: repeatedly select the nearest hit after the last committed one
    while (!sink.finished(a.M)) {
      float bt = INFINITY, ba = 0.f;
      int br = 0x7fffffff, bp = -1;
      for (int j = c.b; j < c.e; ++j) {
        const uint64_t key = a.keys[j];
        if (__uint_as_float((uint32_t)(key >> 32)) > bt) break;
        const int rj = (int)(uint32_t)key;
        const Rec& rec = a.recs[rj];
        if (c.px < rec.px0 || c.px > rec.px1 || c.py < rec.py0 || c.py > rec.py1) continue;
        const PairGeom g = eval_pair(rec, c.u, c.v, c.eps, (double)a.z_near, delta);
        if (!g.ok) continue;
        const float t32 = (float)g.t;
        if (key_less(lt, lr, t32, rj) && key_less(t32, rj, bt, br)) {
          bt = t32; br = rj; bp = j - c.b;
          ba = (float)g.a;
        }
      }
      if (bp < 0) break;
      sink.commit(a, c, bt, br, ba, bp);
      lt = bt; lr = br;
    }
  }
}

// ------------------------------------------------------------------ forward
struct FwdSink {
  float T, D, N0, N1, N2;
  int count;
  float lam5;
  int mode;
  __device__ bool finished(int M) const { return T == 0.f || count >= M; }
  __device__ void commit(const RenderArgs& a, const ItemCtx&, float t, int r, float as, int) {
    const Rec& rec = a.recs[r];
    float omw;
    const float w = splat_weight(as, lam5, mode, omw);
    const float Tw = T * w;
    D = fmaf(Tw, t, D);                 // Eq. 11
    N0 = fmaf(Tw, rec.nx, N0);          // Eq. 12
    N1 = fmaf(Tw, rec.ny, N1);
    N2 = fmaf(Tw, rec.nz, N2);
    T = T * omw;                        // Eq. 13
    ++count;
  }
};

template <int P>
__global__ __launch_bounds__(64) void render_fwd_kernel(RenderArgs a) {
  if (a.counters[C_OVERFLOW]) return;
  ItemCtx c;
  if (item_setup(a, blockIdx.x, c) != 0) return;
  const float lam = a.lambda[0];
  const float lam5 = 5.f * lam;
  const double delta = fringe_margin((double)lam, (double)a.tau, a.mode);
  FwdSink s{1.f, 0.f, 0.f, 0.f, 0.f, 0, lam5, a.mode};
  walk<P>(a, c, s, lam5, delta);
  if (c.inimg) {
    a.depth[c.pix] = s.D;
    if (a.trans) a.trans[c.pix] = s.T;
    if (a.count) a.count[c.pix] = s.count;
    const int64_t nb = 3 * c.pix_off + (c.pix - c.pix_off);
    a.normal[nb] = s.N0;
    a.normal[nb + c.HW] = s.N1;
    a.normal[nb + 2 * c.HW] = s.N2;
  }
}

// ------------------------------------------------------------------ backward
constexpr int kChunk = 12;   // hits per lane kept in LDS per recompute pass

struct BwdLds {
  int pos[kChunk][64];
  float a[kChunk][64];    // a* of the hit
  float T[kChunk][64];    // transmittance in front of the hit
  float cg[kChunk][64];   // c_j, then dL/dw_j after the back-to-front walk
};

struct BwdSink {
  float T;
  int count;
  int c0;
  float Ttail, Stail;
  float gD, gN0, gN1, gN2;
  float lam5;
  int mode;
  BwdLds* L;
  __device__ bool finished(int M) const { return T == 0.f || count >= M; }
  __device__ void commit(const RenderArgs& a, const ItemCtx&, float t, int r, float as, int pos) {
    const Rec& rec = a.recs[r];
    float omw;
    const float w = splat_weight(as, lam5, mode, omw);
    const float cv = gD * t + (gN0 * rec.nx + gN1 * rec.ny + gN2 * rec.nz);
    const int j = count - c0;
    const int lane = threadIdx.x;
    if (j >= 0 && j < kChunk) {
      L->pos[j][lane] = pos;
      L->a[j][lane] = as;
      L->T[j][lane] = T;
      L->cg[j][lane] = cv;
    } else if (j >= kChunk) {
      Stail = fmaf(Ttail * w, cv, Stail);
      Ttail = Ttail * omw;
    }
    T = T * omw;
    ++count;
  }
};

template <int P>
__global__ __launch_bounds__(64) void render_bwd_kernel(RenderArgs a) {
  __shared__ BwdLds L;
  if (a.counters[C_OVERFLOW]) return;
  ItemCtx c;
  const int st = item_setup(a, blockIdx.x, c);
  if (st == 2) return;
  const int lane = threadIdx.x;
  // clear this block's partial rows of the tile list (blocks outside the
  // image too: the per-record sums read every block of a tile)
  for (int i = lane; i < c.e - c.b; i += 64) {
    float4* row = (float4*)(a.partial + ((size_t)a.emit[c.b + i] * a.max_sub + c.sub) * 16);
    const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
    row[0] = z; row[1] = z; row[2] = z; row[3] = z;
  }
  __threadfence_block();
  if (st == 1) return;
  const float lam = a.lambda[0];
  const float lam5 = 5.f * lam;
  const double delta = fringe_margin((double)lam, (double)a.tau, a.mode);
  float gD = 0.f, gN0 = 0.f, gN1 = 0.f, gN2 = 0.f;
  if (c.inimg) {
    gD = a.g_depth[c.pix];
    const int64_t nb = 3 * c.pix_off + (c.pix - c.pix_off);
    gN0 = a.g_normal[nb];
    gN1 = a.g_normal[nb + c.HW];
    gN2 = a.g_normal[nb + 2 * c.HW];
  }
  int passes = 1;
  for (int pass = 0; pass < passes; ++pass) {
    BwdSink s{1.f, 0, pass * kChunk, 1.f, 0.f, gD, gN0, gN1, gN2, lam5, a.mode, &L};
    walk<P>(a, c, s, lam5, delta);
    if (pass == 0) {
      const int jmax = wave_max_int(s.count);
      passes = (jmax + kChunk - 1) / kChunk;
      if (passes > 1 && lane == 0)
        atomicAdd((unsigned long long*)&a.counters[C_BWD_PASSES], (unsigned long long)(passes - 1));
    }
    // back-to-front walk over this chunk
    const int nE = max(0, min(kChunk, s.count - pass * kChunk));
    float S = s.Stail;
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
    // visit the chunk's candidates in list order
    int k = 0;
    int npos = nE > 0 ? L.pos[0][lane] : 0x7fffffff;
    while (true) {
      const int p = uniform_int(wave_min_int(npos));
      if (p == 0x7fffffff) break;
      const uint64_t key = a.keys[c.b + p];
      const int ri = (int)(uint32_t)key;
      const Rec& rec = a.recs[ri];
      const bool act = npos == p;
      float A[13];
#pragma unroll
      for (int q = 0; q < 13; ++q) A[q] = 0.f;
      if (act) {
        const float T = L.T[k][lane], gw = L.cg[k][lane];
        const PairGeom g = eval_pair(rec, c.u, c.v, c.eps, (double)a.z_near, delta);
        const float t = (float)g.t, a32 = (float)g.a;
        const float PX = (float)g.PX, PY = (float)g.PY, den = (float)g.den;
        float omw;
        const float w = splat_weight(a32, lam5, a.mode, omw);
        const float Tw = T * w;
        const float ga = gw * splat_weight_grad(a32, w, omw, lam5, a.mode);
        const float gaX = g.xbranch ? ga : 0.f, gaY = g.xbranch ? 0.f : ga;
        const bool xp = g.PX > 0.0, yp = g.PY > 0.0;
        const float gPX = xp ? -gaX : gaX;
        const float gPY = yp ? -gaY : gaY;
        // d.vx = (P_X + (p - o).vx) / t, d.vy likewise (x = o + t d)
        const float it = 1.f / t;
        const float G = Tw * gD + (gPX * (PX + rec.pvx) + gPY * (PY + rec.pvy)) * it;
        const float Gd = G / den;
        A[0] = gPX;
        A[1] = gPY;
        A[2] = Gd;
        A[3] = gPX * PY - gPY * PX;
        A[4] = Gd * PX;
        A[5] = Gd * PY;
        A[6] = Tw * gN0;
        A[7] = Tw * gN1;
        A[8] = Tw * gN2;
        A[9] = xp ? gaX : 0.f;
        A[10] = xp ? 0.f : gaX;
        A[11] = yp ? gaY : 0.f;
        A[12] = yp ? 0.f : gaY;
      }
#pragma unroll
      for (int q = 0; q < 13; ++q) A[q] = wave_sum(A[q]);
      if (lane == 0) {
        float* row = a.partial + ((size_t)a.emit[c.b + p] * a.max_sub + c.sub) * 16;
#pragma unroll
        for (int q = 0; q < 13; ++q) row[q] += A[q];
      }
      if (act) {
        ++k;
        npos = k < nE ? L.pos[k][lane] : 0x7fffffff;
      }
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
__global__ __launch_bounds__(64) void bwd_reduce_kernel(RenderArgs a) {
  const int k = blockIdx.x;
  if (k >= a.K) return;
  const int lane = threadIdx.x;
  double gp[3] = {0, 0, 0}, gw[3] = {0, 0, 0}, gr[4] = {0, 0, 0, 0};
  double qn[4] = {0, 0, 0, 0}, qnorm = 0;
  const bool ok = !a.counters[C_OVERFLOW];
  for (int s = 0; s < a.S && ok; ++s) {
    const ps_slot sl = a.slots[s];
    if (k < sl.plane_begin || k >= sl.plane_end) continue;
    if (sl.cam < 0 || sl.cam >= a.n_cams) continue;
    const int r = sl.rec_begin + (k - sl.plane_begin);
    if (a.recs[r].cull) continue;
    const int nsub = (sl.tile_w >> 3) * (sl.tile_h >> 3);
    const int rows = a.rec_cnt[r] * nsub;
    const int e0 = a.rec_off[r];
    float A[13];
#pragma unroll
    for (int q = 0; q < 13; ++q) A[q] = 0.f;
    for (int idx = lane; idx < rows; idx += 64) {
      const int e = e0 + idx / nsub, sb = idx % nsub;
      const float4* row = (const float4*)(a.partial + ((size_t)e * a.max_sub + sb) * 16);
      const float4 r0 = row[0], r1 = row[1], r2 = row[2], r3 = row[3];
      A[0] += r0.x; A[1] += r0.y; A[2] += r0.z; A[3] += r0.w;
      A[4] += r1.x; A[5] += r1.y; A[6] += r1.z; A[7] += r1.w;
      A[8] += r2.x; A[9] += r2.y; A[10] += r2.z; A[11] += r2.w;
      A[12] += r3.x;
    }
#pragma unroll
    for (int q = 0; q < 13; ++q) A[q] = wave_sum(A[q]);
    const ps_camera cam = a.cams[sl.cam];
    Frame f;
    if (!plane_frame(a.center, a.quat, k, cam, f)) continue;
    for (int q = 0; q < 4; ++q) qn[q] = f.q[q];
    qnorm = f.qnorm;
    const double sg = a.two_sided ? (f.h > 0.0 ? -1.0 : 1.0) : 1.0;
    double gs[3];   // s R^T dL/d(rendered normal)
    for (int i = 0; i < 3; ++i)
      gs[i] = sg * ((double)cam.R[i] * A[6] + (double)cam.R[3 + i] * A[7] + (double)cam.R[6 + i] * A[8]);
    const double nxg[3] = {f.n[1] * gs[2] - f.n[2] * gs[1], f.n[2] * gs[0] - f.n[0] * gs[2],
                           f.n[0] * gs[1] - f.n[1] * gs[0]};
    for (int i = 0; i < 3; ++i) {
      gp[i] += (double)A[2] * f.n[i] - (double)A[0] * f.vx[i] - (double)A[1] * f.vy[i];
      gw[i] += (double)A[3] * f.n[i] + (double)A[5] * f.vx[i] - (double)A[4] * f.vy[i] + nxg[i];
    }
    for (int q = 0; q < 4; ++q) gr[q] += A[9 + q];
  }
  if (lane == 0) {
    for (int i = 0; i < 3; ++i) a.g_center[3 * k + i] = (float)gp[i];
    for (int q = 0; q < 4; ++q) a.g_radii[4 * k + q] = (float)gr[q];
    // 2 (0, w) (x) q^  =  2 (-(w . v), q0 w + w x v),  v = (q1, q2, q3)
    float gq[4] = {0.f, 0.f, 0.f, 0.f};
    if (qnorm > 0) {
      const double s2 = 2.0 / qnorm;
      const double v0 = qn[1], v1 = qn[2], v2 = qn[3];
      gq[0] = (float)(s2 * -(gw[0] * v0 + gw[1] * v1 + gw[2] * v2));
      gq[1] = (float)(s2 * (qn[0] * gw[0] + (gw[1] * v2 - gw[2] * v1)));
      gq[2] = (float)(s2 * (qn[0] * gw[1] + (gw[2] * v0 - gw[0] * v2)));
      gq[3] = (float)(s2 * (qn[0] * gw[2] + (gw[0] * v1 - gw[1] * v0)));
    }
    for (int q = 0; q < 4; ++q) a.g_quat[4 * k + q] = gq[q];
  }
}

constexpr int kPending = 6;

int fill_args(const ps_layout* L, void* ws, const ps_camera* cams, int n_cams, const float* lambda,
              const ps_params* prm, RenderArgs& a, const char* who) {
  int rc = ps_check_ws(L, ws, who);
  if (rc) return rc;
  if (!cams || !lambda || !prm) return ps_set_error(PS_ERR_INVALID, "%s: null pointer", who);
  if (n_cams <= 0) return ps_set_error(PS_ERR_INVALID, "%s: n_cams <= 0", who);
  if (!(prm->tau > 0.f && prm->tau < 1.f) || !(prm->z_near > 0.f) || prm->M < 1 || prm->M > kMaxM ||
      (prm->weight_mode != 0 && prm->weight_mode != 1))
    return ps_set_error(PS_ERR_INVALID, "%s: bad ps_params", who);
  char* base = (char*)ws;
  memset(&a, 0, sizeof(a));
  a.slots = (const ps_slot*)(base + L->region[R_SLOTS]);
  a.S = L->n_slots;
  a.n_items = L->n_items;
  a.recs = (const Rec*)(base + L->region[R_REC]);
  a.tile_off = (const int*)(base + L->region[R_TILE_OFF]);
  a.keys = (const uint64_t*)(base + L->region[R_KEYS_S]);
  a.emit = (const uint32_t*)(base + L->region[R_EMIT_S]);
  a.rec_cnt = (const int*)(base + L->region[R_REC_CNT]);
  a.rec_off = (const int*)(base + L->region[R_REC_OFF]);
  a.cams = cams;
  a.n_cams = n_cams;
  a.lambda = lambda;
  a.tau = prm->tau; a.z_near = prm->z_near; a.M = prm->M; a.mode = prm->weight_mode;
  a.flags = prm->flags; a.two_sided = prm->two_sided;
  a.counters = (long long*)(base + L->region[R_COUNTERS]);
  a.partial = (float*)(base + L->region[R_PARTIAL]);
  a.max_sub = L->max_sub;
  return PS_OK;
}

}  // namespace

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
  if (a.n_items == 0) return PS_OK;
  hipLaunchKernelGGL(render_fwd_kernel<kPending>, dim3(a.n_items), dim3(64), 0, (hipStream_t)stream, a);
  PS_HIP_CHECK(hipGetLastError());
  return PS_OK;
}

extern "C" int plane_render_bwd(const ps_layout* L, void* ws, const float* center, const float* quat,
                                const float* radii, int K, const ps_camera* cams, int n_cams,
                                const float* lambda, const ps_params* prm, const float* g_depth,
                                const float* g_normal, float* g_center, float* g_quat, float* g_radii,
                                void* stream) {
  RenderArgs a;
  int rc = fill_args(L, ws, cams, n_cams, lambda, prm, a, "plane_render_bwd");
  if (rc) return rc;
  if (!center || !quat || !radii || !g_depth || !g_normal || !g_center || !g_quat || !g_radii)
    return ps_set_error(PS_ERR_INVALID, "plane_render_bwd: null pointer");
  if (K < L->n_planes) return ps_set_error(PS_ERR_INVALID, "plane_render_bwd: K=%d < planes referenced %d", K, L->n_planes);
  a.g_depth = g_depth; a.g_normal = g_normal;
  a.center = center; a.quat = quat; a.K = K;
  a.g_center = g_center; a.g_quat = g_quat; a.g_radii = g_radii;
  hipStream_t st = (hipStream_t)stream;
  if (a.n_items > 0)
    hipLaunchKernelGGL(render_bwd_kernel<kPending>, dim3(a.n_items), dim3(64), 0, st, a);
  if (K > 0) hipLaunchKernelGGL(bwd_reduce_kernel, dim3(K), dim3(64), 0, st, a);
  PS_HIP_CHECK(hipGetLastError());
  return PS_OK;
}
