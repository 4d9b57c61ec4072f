// tile_bin: (tile, plane) pairs keyed by a per-tile depth lower bound.
//
//   count  (one wave per (record, group of 64 tiles of its tile box)): tiles
//          of the record's footprint that pass a separating-axis test
//          against the projected grown rectangle and have a hit in front of
//          the camera; per-tile counts by atomics.
//   scan   (1024-thread workgroups, one per 4096 tiles and 4096 records):
//          exclusive prefix sums of the chunk's tile and record counts with
//          wave64 shuffles plus one LDS pass, the chunk's list-length
//          histogram and each tile's job slot; the last workgroup to finish
//          scans the chunk totals (the chunk bases, which the later passes
//          add to the chunk-local offsets), turns the histograms into the
//          render items' bucket starts, and checks capacity and per-tile
//          limits.
//   emit   (the units of count): key = (depth bound bits << 32 | record),
//          value = emit index (record-major), scattered into tile segments.
//   sort   (one wave per tile): bitonic sort of the tile's keys, across the
//          lanes for lists of at most 64 entries, in LDS up to kSmallSort;
//          longer lists in a second kernel (1024-thread workgroups, LDS
//          sorts of 4096 entries and merges).  Keys are unique, so the order
//          is deterministic.  The sort also writes the records in list order
//          (one contiguous, coalesced run per tile for the render loops) and
//          the descriptors of the tile's 8x8 render items.
//
// The depth bound of a record over a tile is the larger of (a) the minimum
// camera z of its grown, near-clipped rectangle and (b) the minimum over the
// tile's extreme pixel centers of h / den: den is affine in the pixel, so
// t = h / den is smallest at a corner of the pixel-center rectangle.  It is
// rounded down to float32 and lowered by one ulp, so the float32 depth of
// every hit in the tile is >= its key.  The render loops rely on that to
// commit hits in exact per-ray depth order.
#include "ps_internal.h"

using namespace ps;

int ps_check_ws(const ps_layout* L, const void* ws, const char* who);

namespace {

struct BinArgs {
  const ps_slot* slots;
  int S, R, T;
  const Rec* recs;
  const BinRec* brecs;
  int* rec_cnt;
  int* chunk_cnt;   // [R][CH]
  int CH;           // chunks of 64 tiles per record, maximum over jobs
  int* rec_off;
  int* tile_cnt;
  int* tile_off;
  int* tile_cur;
  uint64_t* keys_u;
  uint32_t* emit_u;
  uint64_t* keys_s;
  uint32_t* emit_s;
  long long* counters;
  int* bigtiles;
  long long capacity;
  Rec* recs_s;        // record copies in sorted order
  ItemDesc* items;
  int* tile_pos;      // first render item of each tile
  int G;              // scan chunks
  int* tbase;         // [G] tile-offset base of each chunk
  int* rbase;         // [G] record-offset base of each chunk
  int* chist;         // [G][kBuckets] render items of each chunk per list-length bucket, then the
                      // chunk's first item position in each bucket
  int* btot;          // [kBuckets] render items per bucket
  int* misc;          // [0] workgroups done, [1] big tiles, [2] largest tile list (zero between calls)
  int* tile_slot;     // [T] job slot of each tile
};

template <bool KEY>
__device__ inline bool tile_test(const Rec& rec, const BinRec& br, const ps_slot& sl, int tx, int ty,
                                 float& key_t) {
  int x0 = tx * sl.tile_w, y0 = ty * sl.tile_h;
  int x1 = min(x0 + sl.tile_w, sl.width) - 1, y1 = min(y0 + sl.tile_h, sl.height) - 1;
  x0 = max(x0, (int)rec.px0); x1 = min(x1, (int)rec.px1);
  y0 = max(y0, (int)rec.py0); y1 = min(y1, (int)rec.py1);
  if (x0 > x1 || y0 > y1) return false;
  const double cu[4] = {x0 + 0.5, x1 + 0.5, x1 + 0.5, x0 + 0.5};
  const double cv[4] = {y0 + 0.5, y0 + 0.5, y1 + 0.5, y1 + 0.5};
  for (int e = 0; e < br.nedge; ++e) {
    // largest signed distance over the pixel-center rectangle: at the corner
    // picked by the signs of the edge normal
    const double nx = br.edge[e][0], ny = br.edge[e][1];
    const double m = nx * (nx > 0.0 ? cu[1] : cu[0]) + ny * (ny > 0.0 ? cv[2] : cv[0]) + br.edge[e][2];
    if (m < -1.0) return false;  // every pixel center more than one pixel outside this edge
  }
  double tmin = 1e300;
  bool any = false;
  for (int c = 0; c < 4; ++c) {
    const double den = fma(rec.Du, cu[c], fma(rec.Dv, cv[c], rec.D0));
    if (rec.h * den > 0.0) {
      // h / den to within a few float64 roundoffs, far below the float32
      // rounding and the one-ulp step below
      if (KEY) tmin = fmin(tmin, rec.h * rcp64(den));
      any = true;
    }
  }
  if (!any) return false;
  if (!KEY) return true;
  const float f = __double2float_rd(fmax((double)br.tlb, tmin));
  key_t = __uint_as_float(__float_as_uint(f) - 1u);  // f > 0: one ulp towards zero
  return true;
}

// Work units of the count and emit passes: (record, group of 64 tiles of its
// tile box, row-major); the 64 lanes of a wave test one group.  The
// workgroups (x, y), y < gridDim.y, take the kRecPerWG records from
// kRecPerWG x on and deal their units round-robin to their kRecPerWG x
// gridDim.y waves, so a record with a large box (a plane near the camera, a
// wide fringe at small lambda) spreads over many waves, and records without
// tiles cost no waves of their own.  The host sets gridDim.y from the record
// count: few records (one scene, where the visible ones with large boxes are
// neighbours in record order) get up to eight times the waves; many (a batch
// of scenes, most records outside their job's view) get one wave per record.
constexpr int kRecPerWG = 8;
inline int unit_split(int R) { return std::max(1, std::min(8, 16384 / std::max(R, 1))); }

// Units of the workgroup's records: ub[i] = first unit of record i, ub[8] the
// total; us[i] = the record's job slot (so a unit's loads do not wait on each
// other).
__device__ inline void unit_bases(const BinArgs& a, int* ub, int* us) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = blockIdx.x * kRecPerWG + w;
  if (lane == 0) {
    int ng = 0, sl = 0;
    if (r < a.R) {
      const BinRec& br = a.brecs[r];
      if (br.nedge != 0) ng = ((br.tx1 - br.tx0 + 1) * (br.ty1 - br.ty0 + 1) + 63) >> 6;
      sl = br.slot;
    }
    ub[1 + w] = ng;
    us[w] = sl;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    ub[0] = 0;
    for (int i = 1; i <= kRecPerWG; ++i) ub[i] += ub[i - 1];
  }
  __syncthreads();
}

// Record (index in the workgroup) of unit u.
__device__ inline int unit_record(const int* ub, int u) {
  int i = 0;
  while (u >= ub[i + 1]) ++i;
  return i;
}

__global__ __launch_bounds__(64 * kRecPerWG) void bin_count_kernel(BinArgs a) {
  __shared__ int ub[kRecPerWG + 1], us[kRecPerWG];
  unit_bases(a, ub, us);
  const int lane = threadIdx.x & 63;
  for (int u = (int)blockIdx.y * kRecPerWG + (threadIdx.x >> 6); u < ub[kRecPerWG]; u += kRecPerWG * gridDim.y) {
    // wave-uniform: the record's fields come in through scalar loads
    const int i = __builtin_amdgcn_readfirstlane(unit_record(ub, u));
    const int r = blockIdx.x * kRecPerWG + i, ch = u - __builtin_amdgcn_readfirstlane(ub[i]);
    const BinRec& br = a.brecs[r];
    const Rec& rec = a.recs[r];
    const ps_slot& sl = a.slots[__builtin_amdgcn_readfirstlane(us[i])];
    const int nx = br.tx1 - br.tx0 + 1;
    const int n = nx * (br.ty1 - br.ty0 + 1);
    const int idx = ch * 64 + lane;
    bool pass = false;
    if (idx < n) {
      const int tx = br.tx0 + idx % nx, ty = br.ty0 + idx / nx;
      float kt;
      pass = tile_test<false>(rec, br, sl, tx, ty, kt);
      if (pass) atomicAdd(&a.tile_cnt[sl.tile_begin + ty * sl.tiles_x + tx], 1);
    }
    const int cnt = __popcll(ballot(pass));
    if (lane == 0) {
      a.chunk_cnt[(size_t)r * a.CH + ch] = cnt;
      if (cnt) atomicAdd(&a.rec_cnt[r], cnt);
    }
  }
}

// Exclusive scan of a chunk of n <= 4096 values by one 1024-thread
// workgroup, thread i holding values 4 i .. 4 i + 3 (zeros past n): writes
// the chunk-local offsets to out and returns the total (and the maximum).
__device__ inline int chunk_scan(const int (&v)[4], int* __restrict__ out, int n, int* lds, int& mx) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  int local = 0;
  for (int j = 0; j < 4; ++j) {
    mx = max(mx, v[j]);
    local += v[j];
  }
  int incl = local;
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) lds[wid] = incl;
  __syncthreads();
  if (wid == 0) {
    const int x = lane < 16 ? lds[lane] : 0;
    int xi = x;
    for (int o = 1; o < 16; o <<= 1) {
      const int y = __shfl_up(xi, o, 64);
      if (lane >= o) xi += y;
    }
    if (lane < 16) lds[16 + lane] = xi - x;
    if (lane == 15) lds[32] = xi;
  }
  __syncthreads();
  int run = lds[16 + wid] + (incl - local);
  for (int j = 0; j < 4; ++j) {
    const int idx = tid * 4 + j;
    if (idx < n) out[idx] = run;
    run += v[j];
  }
  const int total = lds[32];
  __syncthreads();
  return total;
}

// Exclusive scan in place of x[0, n), int32 values that other workgroups
// wrote (read with device-scope loads), by one 1024-thread workgroup, 1024
// values at a time; returns the total.  lsum: 17 int64 of LDS.
__device__ inline long long block_scan_inplace(int* x, int n, long long* lsum) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  long long carry = 0;
  for (int b0 = 0; b0 < n; b0 += 1024) {
    const int i = b0 + tid;
    const long long v = i < n ? __hip_atomic_load(&x[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
    long long incl = v;
    for (int o = 1; o < 64; o <<= 1) {
      const long long y = __shfl_up(incl, o, 64);
      if (lane >= o) incl += y;
    }
    if (lane == 63) lsum[wid] = incl;
    __syncthreads();
    if (tid == 0) {
      long long run = 0;
      for (int w = 0; w < 16; ++w) {
        const long long t = lsum[w];
        lsum[w] = run;
        run += t;
      }
      lsum[16] = run;
    }
    __syncthreads();
    if (i < n) x[i] = (int)(carry + lsum[wid] + incl - v);
    carry += lsum[16];
    __syncthreads();
  }
  return carry;
}

// Job slots are cached in LDS for the tile-to-slot search when there are at
// most this many
constexpr int kSlotCache = 1024;

__global__ __launch_bounds__(1024) void bin_scan_kernel(BinArgs a) {
  __shared__ int lds[40];
  __shared__ int hist[kBuckets];
  __shared__ int stb[kSlotCache];   // tile_begin of each slot
  __shared__ int ssub[kSlotCache];  // 8x8 blocks per tile of each slot
  __shared__ long long lsum[17];
  __shared__ int last;
  const int g = blockIdx.x, tid = threadIdx.x;
  const int t0 = g * kScanChunk, r0 = g * kScanChunk;
  const int nt = max(0, min(kScanChunk, a.T - t0)), nr = max(0, min(kScanChunk, a.R - r0));
  const bool cached = a.S <= kSlotCache;
  // every load up front: the chunk's tile and record counts (four per
  // thread) and the slots' first tiles and tile shapes
  int vt[4], vr[4];
  for (int j = 0; j < 4; ++j) {
    const int idx = tid * 4 + j;
    vt[j] = idx < nt ? a.tile_cnt[t0 + idx] : 0;
    vr[j] = idx < nr ? a.rec_cnt[r0 + idx] : 0;
  }
  for (int k = tid; k < kBuckets; k += blockDim.x) hist[k] = 0;
  if (cached)
    for (int s = tid; s < a.S; s += blockDim.x) {
      const ps_slot& q = a.slots[s];
      stb[s] = q.tile_begin;
      ssub[s] = (q.tile_w >> 3) * (q.tile_h >> 3);
    }
  int mx_t = 0, mx_r = 0;
  const int tot_t = chunk_scan(vt, a.tile_off + t0, nt, lds, mx_t);
  const int tot_r = chunk_scan(vr, a.rec_off + r0, nr, lds, mx_r);
  // the chunk's render items per list-length bucket: each tile's items take
  // consecutive positions in its bucket after those of the chunk's earlier
  // claims (tile_pos holds the position inside the chunk's share of the
  // bucket; the order of tiles inside a bucket does not matter: items are
  // independent); bin_emit's scatter cursors
  for (int j = 0; j < 4; ++j) {   // the tiles this thread scanned
    const int t = t0 + tid * 4 + j;
    if (t >= t0 + nt) break;
    int si, sub_per;
    if (cached) {   // last slot whose first tile is <= t
      int lo = 0, hi = a.S - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (stb[mid] <= t) lo = mid; else hi = mid - 1;
      }
      si = lo;
      sub_per = ssub[si];
    } else {
      si = find_slot_by_tile(a.slots, a.S, t);
      const ps_slot& sl = a.slots[si];
      sub_per = (sl.tile_w >> 3) * (sl.tile_h >> 3);
    }
    const int c = vt[j];
    a.tile_slot[t] = si;
    a.tile_pos[t] = atomicAdd(&hist[length_bucket(c)], sub_per);
    a.tile_cur[t] = 0;
    if (c > kSmallSort && c <= kMaxList) a.bigtiles[atomicAdd(&a.misc[1], 1)] = t;
  }
  for (int w = 64; w > 1; w >>= 1) mx_t = max(mx_t, __shfl_xor(mx_t, w >> 1, 64));
  __syncthreads();
  for (int k = tid; k < kBuckets; k += blockDim.x) a.chist[(size_t)g * kBuckets + k] = hist[k];
  if ((tid & 63) == 0 && mx_t) atomicMax(&a.misc[2], mx_t);
  if (tid == 0) {
    a.tbase[g] = tot_t;
    a.rbase[g] = tot_r;
  }
  // the last workgroup to finish combines the chunks (a single workgroup is
  // the last: no device-scope fence, which writes back the L2 of the XCD)
  if (gridDim.x > 1) {
    __threadfence();
    __syncthreads();
    if (tid == 0) last = atomicAdd(&a.misc[0], 1) == (int)gridDim.x - 1;
    __syncthreads();
    if (!last) return;
    __threadfence();
  } else {
    __syncthreads();
  }
  // chunk bases: exclusive scans of the chunk totals (one chunk: its own)
  const long long tb = a.G == 1 ? tot_t : block_scan_inplace(a.tbase, a.G, lsum);
  const long long rb = a.G == 1 ? tot_r : block_scan_inplace(a.rbase, a.G, lsum);
  if (tid == 0) {
    if (a.G == 1) {
      a.tbase[0] = 0;
      a.rbase[0] = 0;
    }
    // the totals after the last entries (the offsets before them stay chunk-local)
    a.tile_off[a.T] = (int)tb;
    a.rec_off[a.R] = (int)rb;
  }
  // items per bucket over the chunks; each chunk's counts become its start
  // inside the bucket (chunks in order; 16 loads in flight per thread).  One
  // chunk: its histogram is still in LDS and starts every bucket at 0.
  if (a.G == 1)
    for (int k = tid; k < kBuckets; k += blockDim.x) a.chist[k] = 0;
  for (int k = tid; k < kBuckets && a.G > 1; k += blockDim.x) {
    int run = 0;
    for (int c0 = 0; c0 < a.G; c0 += 16) {
      int v[16];
#pragma unroll
      for (int j = 0; j < 16; ++j)
        v[j] = c0 + j < a.G ? __hip_atomic_load(&a.chist[(size_t)(c0 + j) * kBuckets + k], __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT)
                            : 0;
#pragma unroll
      for (int j = 0; j < 16; ++j)
        if (c0 + j < a.G) {
          a.chist[(size_t)(c0 + j) * kBuckets + k] = run;
          run += v[j];
        }
    }
    hist[k] = run;
  }
  __syncthreads();
  const long long total = tb;   // pairs (beyond int range: flagged as overflow below)
  if (tid < 64) {   // exclusive scan over buckets, longest first: 16 buckets per lane
    const int lane = tid;
    int loc = 0;
    for (int i = 0; i < 16; ++i) loc += hist[kBuckets - 1 - (16 * lane + i)];
    int incl = loc;
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(incl, o, 64);
      if (lane >= o) incl += y;
    }
    int run = incl - loc;
    for (int i = 0; i < 16; ++i) {
      const int k = kBuckets - 1 - (16 * lane + i);
      const int h = hist[k];
      a.btot[k] = run;   // first item position of the bucket
      run += h;
    }
  }
  if (tid == 0) {
    const int mx = __hip_atomic_load(&a.misc[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int nbig = __hip_atomic_load(&a.misc[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    a.misc[0] = 0;
    a.misc[1] = 0;
    a.misc[2] = 0;
    a.counters[C_PAIRS] = total;
    a.counters[C_MAXTILE] = mx;
    a.counters[C_NBIG] = nbig;
    a.counters[C_OVERFLOW] = (total > a.capacity || mx > kMaxList) ? 1 : 0;
    if (a.counters[C_OVERFLOW]) a.counters[C_STICKY] = 1;
    a.counters[C_SLOW] = 0;
    a.counters[C_BWD_PASSES] = 0;
    for (int k = C_EVALS; k < C_STICKY; ++k) a.counters[k] = 0;
    a.counters[C_BT_MAX] = 0;
  }
}

// Work units as in bin_count_kernel: the j-th passing tile of record r, in
// tile-box order, gets emit index rec_off[r] + j (the counts of the earlier
// groups, summed across the lanes, then a ballot prefix count).
__global__ __launch_bounds__(64 * kRecPerWG) void bin_emit_kernel(BinArgs a) {
  __shared__ int ub[kRecPerWG + 1], us[kRecPerWG];
  if (a.counters[C_OVERFLOW]) return;
  unit_bases(a, ub, us);
  const int lane = threadIdx.x & 63;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int u = (int)blockIdx.y * kRecPerWG + (threadIdx.x >> 6); u < ub[kRecPerWG]; u += kRecPerWG * gridDim.y) {
    // wave-uniform: the record's fields come in through scalar loads
    const int i = __builtin_amdgcn_readfirstlane(unit_record(ub, u));
    const int r = blockIdx.x * kRecPerWG + i, ch = u - __builtin_amdgcn_readfirstlane(ub[i]);
    const BinRec& br = a.brecs[r];
    const Rec& rec = a.recs[r];
    const ps_slot& sl = a.slots[__builtin_amdgcn_readfirstlane(us[i])];
    const int nx = br.tx1 - br.tx0 + 1;
    const int n = nx * (br.ty1 - br.ty0 + 1);
    const int* cc = a.chunk_cnt + (size_t)r * a.CH;
    int before = 0;   // passing tiles of the groups before ch
    for (int c = lane; c < ch; c += 64) before += cc[c];
    for (int o = 32; o > 0; o >>= 1) before += __shfl_xor(before, o, 64);
    const int j = a.rec_off[r] + a.rbase[r / kScanChunk] + before;
    const int idx = ch * 64 + lane;
    bool pass = false;
    float kt = 0.f;
    int tx = 0, ty = 0;
    if (idx < n) {
      tx = br.tx0 + idx % nx;
      ty = br.ty0 + idx / nx;
      pass = tile_test<true>(rec, br, sl, tx, ty, kt);
    }
    const uint64_t m = ballot(pass);
    if (pass) {
      const int gt = sl.tile_begin + ty * sl.tiles_x + tx;
      const int slot = a.tile_off[gt] + a.tbase[gt / kScanChunk] + atomicAdd(&a.tile_cur[gt], 1);
      a.keys_u[slot] = ((uint64_t)__float_as_uint(kt) << 32) | (uint32_t)r;
      a.emit_u[slot] = (uint32_t)(j + __popcll(m & below));
    }
  }
}

template <int CAP, int NT>
__device__ void lds_bitonic(uint64_t* k, uint32_t* v, int n, const uint64_t* __restrict__ kin,
                            const uint32_t* __restrict__ vin, uint64_t* __restrict__ kout,
                            uint32_t* __restrict__ vout, const Rec* __restrict__ recs,
                            Rec* __restrict__ rout) {
  int n2 = 1;
  while (n2 < n) n2 <<= 1;
  for (int i = threadIdx.x; i < n2; i += NT) {
    k[i] = i < n ? kin[i] : ~0ull;
    v[i] = i < n ? vin[i] : 0u;
  }
  __syncthreads();
  for (int size = 2; size <= n2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < (n2 >> 1); i += NT) {
        const int lo = ((i / stride) * 2 * stride) + (i % stride);
        const int hi = lo + stride;
        const bool up = (lo & size) == 0;
        const uint64_t a = k[lo], b = k[hi];
        if ((a > b) == up) {
          k[lo] = b; k[hi] = a;
          const uint32_t t = v[lo]; v[lo] = v[hi]; v[hi] = t;
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < n; i += NT) {
    kout[i] = k[i];
    vout[i] = v[i];
  }
  if (!rout) return;
  // record copies in list order, eight lanes per 128-byte record
  for (int i = threadIdx.x; i < 8 * n; i += NT) {
    const int e = i >> 3, q = i & 7;
    const int ri = (int)(uint32_t)k[e];
    reinterpret_cast<float4*>(&rout[e])[q] = reinterpret_cast<const float4*>(&recs[ri])[q];
  }
}

// One wave per tile.  The tile's render items, then its sort: a list of at
// most 64 entries in registers (a bitonic network across the lanes, one key
// per lane), up to kSmallSort in LDS; longer lists are left to
// bin_sort_big_kernel.  The list's keys are fetched before the item
// bookkeeping, so their latency overlaps it.
__global__ __launch_bounds__(64) void bin_sort_small_kernel(BinArgs a) {
  __shared__ uint64_t k[kSmallSort];
  __shared__ uint32_t v[kSmallSort];
  const int t = blockIdx.x, lane = threadIdx.x;
  const int n = a.tile_cnt[t];
  const int off = a.tile_off[t] + a.tbase[t / kScanChunk];   // chunk-local offset + chunk base
  const bool reg = n <= 64;
  uint64_t key = ~0ull;
  uint32_t val = 0u;
  if (reg && lane < n) {
    key = a.keys_u[off + lane];
    val = a.emit_u[off + lane];
  }
  const int s = a.tile_slot[t];
  const ps_slot& sl = a.slots[s];
  const int sub_w = sl.tile_w >> 3;
  const int sub_per = sub_w * (sl.tile_h >> 3);
  // the tile's first render item: its bucket's start + its chunk's start in
  // the bucket + its place among the chunk's tiles of the bucket
  const int kb = length_bucket(n);
  const int pos0 = a.btot[kb] + a.chist[(size_t)(t / kScanChunk) * kBuckets + kb] + a.tile_pos[t];
  if (lane == 0) a.tile_off[t] = off;   // final offset, for bin_sort_big
  // render items (8x8 blocks) of this tile, placed by list length
  if (lane < sub_per) {
    const int sub = lane;
    const int lt = t - sl.tile_begin;
    ItemDesc d;
    d.b = off;
    d.e = off + n;
    d.ox = (int16_t)((lt % sl.tiles_x) * sl.tile_w + (sub % sub_w) * 8);
    d.oy = (int16_t)((lt / sl.tiles_x) * sl.tile_h + (sub / sub_w) * 8);
    d.width = (int16_t)sl.width;
    d.height = (int16_t)sl.height;
    d.cam = sl.cam;
    d.sub = (int16_t)sub;
    d.slot = (int16_t)s;
    d.pix_off = sl.pix_off;
    a.items[pos0 + sub] = d;
  }
  if (a.counters[C_OVERFLOW]) return;
  if (n == 0 || n > kSmallSort) return;
  if (!reg) {
    lds_bitonic<kSmallSort, 64>(k, v, n, a.keys_u + off, a.emit_u + off, a.keys_s + off, a.emit_s + off,
                                a.recs, a.recs_s + off);
    return;
  }
  // bitonic network over the n2 >= n lanes (unused lanes hold the largest
  // key and stay at the end); keys are unique
  int n2 = 1;
  while (n2 < n) n2 <<= 1;
  for (int size = 2; size <= n2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      const uint32_t klo = (uint32_t)key, khi = (uint32_t)(key >> 32);
      const uint64_t ok = ((uint64_t)(uint32_t)__shfl_xor((int)khi, stride, 64) << 32) |
                          (uint32_t)__shfl_xor((int)klo, stride, 64);
      const uint32_t ov = (uint32_t)__shfl_xor((int)val, stride, 64);
      const bool up = (lane & size) == 0;
      const bool lower = (lane & stride) == 0;
      const bool take = lower == up ? ok < key : ok > key;   // keep the smaller in the lower lane when ascending
      if (take) {
        key = ok;
        val = ov;
      }
    }
  }
  if (lane < n) {
    a.keys_s[off + lane] = key;
    a.emit_s[off + lane] = val;
  }
  // record copies in list order, eight lanes per 128-byte record
  const int rec_lo = (int)(uint32_t)key;
  for (int i0 = 0; i0 < 8 * n; i0 += 64) {   // every lane takes part in the exchange
    const int i = i0 + lane, e = i >> 3, q = i & 7;
    const int ri = __shfl(rec_lo, e & 63, 64);
    if (i < 8 * n)
      reinterpret_cast<float4*>(&a.recs_s[off + e])[q] = reinterpret_cast<const float4*>(&a.recs[ri])[q];
  }
}

// One merge pass over a tile list made of sorted runs of length L: the runs
// 2m and 2m + 1 merge into one run of 2L.  Keys are unique (the record index
// is in the low bits), so each entry's place is its index in its own run plus
// the number of smaller keys in the other run (a binary search).
__device__ void merge_pass(const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint64_t* kout,
                           uint32_t* vout, int n, int L) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int r = i / L;
    const int ps = (r & ~1) * L;                  // start of the pair
    const bool first = (r & 1) == 0;
    const int ob = first ? ps + L : ps;           // the other run [ob, oe)
    const int oe = first ? min(ps + 2 * L, n) : ps + L;
    const uint64_t key = kin[i];
    int lo = ob, hi = max(ob, oe);
    while (lo < hi) {                             // first entry of the other run >= key
      const int mid = (lo + hi) >> 1;
      if (kin[mid] < key) lo = mid + 1; else hi = mid;
    }
    const int own = first ? i - ps : i - (ps + L);
    const int o = ps + own + (lo - ob);
    kout[o] = key;
    vout[o] = vin[i];
  }
}

// Tile lists longer than kSmallSort.  Up to kBigSort entries: one bitonic
// sort in LDS.  Longer (to kMaxList): chunks of kBigSort sorted in LDS, then
// merge passes that move the runs between the tile's unsorted and sorted
// segments (both hold n entries), ending in the sorted one.
__global__ __launch_bounds__(1024) void bin_sort_big_kernel(BinArgs a) {
  extern __shared__ unsigned char smem[];
  uint64_t* k = (uint64_t*)smem;
  uint32_t* v = (uint32_t*)(smem + 8 * kBigSort);
  if (a.counters[C_OVERFLOW]) return;
  const int nbig = (int)a.counters[C_NBIG];
  for (int b = blockIdx.x; b < nbig; b += gridDim.x) {
    const int t = a.bigtiles[b];
    const int n = a.tile_cnt[t];
    const int off = a.tile_off[t];
    if (n <= kBigSort) {
      lds_bitonic<kBigSort, 1024>(k, v, n, a.keys_u + off, a.emit_u + off, a.keys_s + off, a.emit_s + off,
                                  a.recs, a.recs_s + off);
      __syncthreads();
      continue;
    }
    // passes needed after the chunk sorts; the chunks go to the segment from
    // which an even number of passes ends in the sorted one
    int passes = 0;
    for (int L = kBigSort; L < n; L <<= 1) ++passes;
    uint64_t* kb[2] = {a.keys_s + off, a.keys_u + off};
    uint32_t* vb[2] = {a.emit_s + off, a.emit_u + off};
    int cur = passes & 1;
    for (int c0 = 0; c0 < n; c0 += kBigSort) {
      const int m = min(kBigSort, n - c0);
      // unsorted input chunk and its output: in place when cur == 1 (the
      // chunk is read into LDS before it is written back)
      lds_bitonic<kBigSort, 1024>(k, v, m, a.keys_u + off + c0, a.emit_u + off + c0, kb[cur] + c0, vb[cur] + c0,
                                  nullptr, nullptr);
      __syncthreads();
    }
    __threadfence_block();
    for (int L = kBigSort; L < n; L <<= 1) {
      merge_pass(kb[cur], vb[cur], kb[cur ^ 1], vb[cur ^ 1], n, L);
      cur ^= 1;
      __threadfence_block();
      __syncthreads();
    }
    // record copies in list order
    for (int i = threadIdx.x; i < 8 * n; i += blockDim.x) {
      const int e = i >> 3, q = i & 7;
      const int ri = (int)(uint32_t)a.keys_s[off + e];
      reinterpret_cast<float4*>(&a.recs_s[off + e])[q] = reinterpret_cast<const float4*>(&a.recs[ri])[q];
    }
    __syncthreads();
  }
}

}  // namespace

extern "C" int tile_bin(const ps_layout* L, void* ws, int64_t* pairs_needed, void* stream) {
  int rc = ps_check_ws(L, ws, "tile_bin");
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  char* base = (char*)ws;
  BinArgs a;
  a.slots = (const ps_slot*)(base + L->region[R_SLOTS]);
  a.S = L->n_slots; a.R = L->n_records; a.T = L->n_tiles;
  a.recs = (const Rec*)(base + L->region[R_REC]);
  a.brecs = (const BinRec*)(base + L->region[R_BINREC]);
  a.rec_cnt = (int*)(base + L->region[R_REC_CNT]);
  a.chunk_cnt = (int*)(base + L->region[R_CHUNK_CNT]);
  a.CH = L->max_chunks;
  a.rec_off = (int*)(base + L->region[R_REC_OFF]);
  a.tile_cnt = (int*)(base + L->region[R_TILE_CNT]);
  a.tile_off = (int*)(base + L->region[R_TILE_OFF]);
  a.tile_cur = (int*)(base + L->region[R_TILE_CUR]);
  a.keys_u = (uint64_t*)(base + L->region[R_KEYS_U]);
  a.emit_u = (uint32_t*)(base + L->region[R_EMIT_U]);
  a.keys_s = (uint64_t*)(base + L->region[R_KEYS_S]);
  a.emit_s = (uint32_t*)(base + L->region[R_EMIT_S]);
  a.counters = (long long*)(base + L->region[R_COUNTERS]);
  a.bigtiles = (int*)(base + L->region[R_BIGTILES]);
  a.capacity = L->pair_capacity;
  a.recs_s = (Rec*)(base + L->region[R_RECS_S]);
  a.items = (ItemDesc*)(base + L->region[R_ITEMS]);
  a.tile_pos = (int*)(base + L->region[R_TILEPOS]);
  a.G = scan_chunks(a.T, a.R);
  a.tbase = (int*)(base + L->region[R_SCAN]);
  a.rbase = a.tbase + a.G;
  a.chist = a.rbase + a.G;
  a.btot = a.chist + (size_t)a.G * kBuckets;
  a.misc = a.btot + kBuckets;
  a.tile_slot = (int*)(base + L->region[R_TILESLOT]);
  // the record and tile counts were cleared by plane_project
  if (a.R > 0)
    hipLaunchKernelGGL(bin_count_kernel, dim3((a.R + kRecPerWG - 1) / kRecPerWG, unit_split(a.R)),
                       dim3(64 * kRecPerWG), 0, st, a);
  hipLaunchKernelGGL(bin_scan_kernel, dim3(a.G), dim3(1024), 0, st, a);
  if (a.R > 0)
    hipLaunchKernelGGL(bin_emit_kernel, dim3((a.R + kRecPerWG - 1) / kRecPerWG, unit_split(a.R)),
                       dim3(64 * kRecPerWG), 0, st, a);
  hipLaunchKernelGGL(bin_sort_small_kernel, dim3(a.T), dim3(64), 0, st, a);
  hipLaunchKernelGGL(bin_sort_big_kernel, dim3(64), dim3(1024), 12 * kBigSort, st, a);
  PS_HIP_CHECK(hipGetLastError());
  if (pairs_needed) {
    long long c[2];
    PS_HIP_CHECK(hipMemcpyAsync(c, a.counters, sizeof(c), hipMemcpyDeviceToHost, st));
    PS_HIP_CHECK(hipStreamSynchronize(st));
    *pairs_needed = c[C_PAIRS];
    if (c[C_OVERFLOW]) {
      if (c[C_PAIRS] > L->pair_capacity)
        return ps_set_error(PS_ERR_CAPACITY, "tile_bin: %lld pairs exceed capacity %lld",
                            (long long)c[C_PAIRS], (long long)L->pair_capacity);
      return ps_set_error(PS_ERR_CAPACITY, "tile_bin: a tile holds more than %d pairs; use smaller tiles",
                          kMaxList);
    }
  }
  return PS_OK;
}
