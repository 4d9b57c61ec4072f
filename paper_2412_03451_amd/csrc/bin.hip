// tile_bin: (tile, plane) pairs keyed by a per-tile depth lower bound.
//
//   count  (one wave per record): tiles of the record's footprint that pass
//          a separating-axis test against the projected grown rectangle and
//          have a hit in front of the camera; per-tile counts by atomics.
//   scan   (1024-thread workgroups, one per 4096 tiles and 4096 records):
//          exclusive prefix sums of the chunk's tile and record counts with
//          wave64 shuffles plus one LDS pass, and the chunk's list-length
//          histogram; the last workgroup to finish scans the chunk totals
//          (the chunk bases, which the later passes add to the chunk-local
//          offsets), turns the histogram into the render items' bucket
//          starts, and checks capacity and per-tile limits.
//   emit   (one wave per record): key = (depth bound bits << 32 | record),
//          value = emit index (record-major), scattered into tile segments.
//   sort   (one workgroup per tile): bitonic sort of the tile's keys in LDS;
//          keys are unique, so the order is deterministic.  The sort also
//          writes the records in list order (one contiguous, coalesced run
//          per tile for the render loops) and the descriptors of the tile's
//          8x8 render items.
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

// One wave per record: the 64 lanes test the record's candidate tiles in
// row-major order, 64 at a time (a plane near the camera can cover every
// tile of the image, so one thread per record would serialise it).
// Waves over (record, group of 64 tiles of its tile box): grid (R / 4, G),
// wave (r, y) takes the groups y, y + G, ... of record r, so records with big
// boxes (planes close to the camera, wide fringes at small lambda) spread
// over up to G waves instead of one long loop.  Each group's count goes to
// chunk_cnt for the emit pass; rec_cnt (cleared with the tile counts)
// accumulates the record's total.
constexpr int kChunkWaves = 8;

__global__ __launch_bounds__(256) void bin_count_kernel(BinArgs a) {
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (r >= a.R) return;
  const BinRec& br = a.brecs[r];
  if (br.nedge == 0) return;
  const int nx = br.tx1 - br.tx0 + 1;
  const int n = nx * (br.ty1 - br.ty0 + 1);
  if ((int)blockIdx.y * 64 >= n) return;
  const Rec& rec = a.recs[r];
  const ps_slot& sl = a.slots[br.slot];
  int total = 0;
  for (int ch = blockIdx.y; ch * 64 < n; ch += gridDim.y) {
    const int idx = ch * 64 + lane;
    bool pass = false;
    if (idx < n) {
      const int tx = br.tx0 + idx % nx, ty = br.ty0 + idx / nx;
      float kt;
      pass = tile_test<false>(rec, br, sl, tx, ty, kt);
      if (pass) atomicAdd(&a.tile_cnt[sl.tile_begin + ty * sl.tiles_x + tx], 1);
    }
    const int cnt = __popcll(ballot(pass));
    if (lane == 0) a.chunk_cnt[(size_t)r * a.CH + ch] = cnt;
    total += cnt;
  }
  if (lane == 0 && total) atomicAdd(&a.rec_cnt[r], total);
}

// Exclusive scan of in[0, n) by one 1024-thread workgroup (n <= 4096):
// chunk-local offsets; returns the total and the maximum.
__device__ inline int chunk_scan(const int* __restrict__ in, int* __restrict__ out, int n, int* lds, int& mx) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  int v[4];
  int local = 0;
  for (int j = 0; j < 4; ++j) {
    const int idx = tid * 4 + j;
    v[j] = idx < n ? in[idx] : 0;
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

__global__ __launch_bounds__(1024) void bin_scan_kernel(BinArgs a) {
  __shared__ int lds[40];
  __shared__ int hist[kBuckets];
  __shared__ int last;
  const int g = blockIdx.x, tid = threadIdx.x;
  const int t0 = g * kScanChunk, r0 = g * kScanChunk;
  const int nt = max(0, min(kScanChunk, a.T - t0)), nr = max(0, min(kScanChunk, a.R - r0));
  for (int k = tid; k < kBuckets; k += blockDim.x) hist[k] = 0;
  int mx_t = 0, mx_r = 0;
  const int tot_t = chunk_scan(a.tile_cnt + t0, a.tile_off + t0, nt, lds, mx_t);
  const int tot_r = chunk_scan(a.rec_cnt + r0, a.rec_off + r0, nr, lds, mx_r);
  // the chunk's render items per list-length bucket: each tile's items take
  // consecutive positions in its bucket after those of the chunk's earlier
  // claims (tile_pos holds the position inside the chunk's share of the
  // bucket; the order of tiles inside a bucket does not matter: items are
  // independent); bin_emit's scatter cursors
  for (int t = t0 + tid; t < t0 + nt; t += blockDim.x) {
    const ps_slot& sl = a.slots[find_slot_by_tile(a.slots, a.S, t)];
    const int sub_per = (sl.tile_w >> 3) * (sl.tile_h >> 3);
    const int c = a.tile_cnt[t];
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
  long long total = 0;
  if (tid == 0) {   // chunk bases (a few hundred chunks at most: in order on one thread)
    long long tb = 0, rb = 0;
    for (int k = 0; k < a.G; ++k) {
      const int ct = __hip_atomic_load(&a.tbase[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const int cr = __hip_atomic_load(&a.rbase[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      a.tbase[k] = (int)tb;
      a.rbase[k] = (int)rb;
      tb += ct;
      rb += cr;
    }
    lds[34] = (int)(tb >> 31);   // pairs beyond int range: flagged as overflow below
    lds[35] = (int)(tb & 0x7fffffff);
    // the totals after the last entries (the offsets before them stay chunk-local)
    a.tile_off[a.T] = (int)tb;
    a.rec_off[a.R] = (int)rb;
  }
  // items per bucket over the chunks; each chunk's counts become its start
  // inside the bucket (chunks in order)
  for (int k = tid; k < kBuckets; k += blockDim.x) {
    int run = 0;
    for (int c = 0; c < a.G; ++c) {
      int* h = &a.chist[(size_t)c * kBuckets + k];
      const int v = __hip_atomic_load(h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      *h = run;
      run += v;
    }
    hist[k] = run;
  }
  __syncthreads();
  total = ((long long)lds[34] << 31) | lds[35];
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

// Waves over (record, group of 64 tiles) as in bin_count_kernel: the j-th
// passing tile of record r, in tile-box order, gets emit index rec_off[r] + j
// (counts of the earlier groups, then a ballot prefix count).
__global__ __launch_bounds__(256) void bin_emit_kernel(BinArgs a) {
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (r >= a.R) return;
  if (a.counters[C_OVERFLOW]) return;
  const BinRec& br = a.brecs[r];
  if (br.nedge == 0) return;
  const int nx = br.tx1 - br.tx0 + 1;
  const int n = nx * (br.ty1 - br.ty0 + 1);
  if ((int)blockIdx.y * 64 >= n) return;
  const Rec& rec = a.recs[r];
  const ps_slot& sl = a.slots[br.slot];
  const int* cc = a.chunk_cnt + (size_t)r * a.CH;
  int j = a.rec_off[r] + a.rbase[r / kScanChunk];
  int done = 0;   // groups counted into j
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int ch = blockIdx.y; ch * 64 < n; ch += gridDim.y) {
    for (; done < ch; ++done) j += cc[done];
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

__global__ __launch_bounds__(256) void bin_sort_small_kernel(BinArgs a) {
  __shared__ uint64_t k[kSmallSort];
  __shared__ uint32_t v[kSmallSort];
  __shared__ int pos0;
  const int t = blockIdx.x;
  const int n = a.tile_cnt[t];
  const int off = a.tile_off[t] + a.tbase[t / kScanChunk];   // chunk-local offset + chunk base
  const int s = find_slot_by_tile(a.slots, a.S, t);
  const ps_slot& sl = a.slots[s];
  const int sub_w = sl.tile_w >> 3;
  const int sub_per = sub_w * (sl.tile_h >> 3);
  // the tile's first render item: its bucket's start + its chunk's start in
  // the bucket + its place among the chunk's tiles of the bucket
  if (threadIdx.x == 0) {
    const int k = length_bucket(n);
    pos0 = a.btot[k] + a.chist[(size_t)(t / kScanChunk) * kBuckets + k] + a.tile_pos[t];
  }
  __syncthreads();
  if (threadIdx.x == 0) a.tile_off[t] = off;   // final offset, for bin_sort_big
  // render items (8x8 blocks) of this tile, placed by list length
  if (threadIdx.x < 16) {
    const int sub = threadIdx.x;
    if (sub < sub_per) {
      const int pos = pos0 + sub;
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
      a.items[pos] = d;
    }
  }
  if (a.counters[C_OVERFLOW]) return;
  if (n == 0 || n > kSmallSort) return;
  lds_bitonic<kSmallSort, 256>(k, v, n, a.keys_u + off, a.emit_u + off, a.keys_s + off, a.emit_s + off,
                               a.recs, a.recs_s + off);
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
  // the record and tile counts were cleared by plane_project
  if (a.R > 0)
    hipLaunchKernelGGL(bin_count_kernel, dim3((a.R + 3) / 4, std::min(a.CH, kChunkWaves)), dim3(256), 0, st, a);
  hipLaunchKernelGGL(bin_scan_kernel, dim3(a.G), dim3(1024), 0, st, a);
  if (a.R > 0)
    hipLaunchKernelGGL(bin_emit_kernel, dim3((a.R + 3) / 4, std::min(a.CH, kChunkWaves)), dim3(256), 0, st, a);
  hipLaunchKernelGGL(bin_sort_small_kernel, dim3(a.T), dim3(256), 0, st, a);
  hipLaunchKernelGGL(bin_sort_big_kernel, dim3(32), dim3(1024), 12 * kBigSort, st, a);
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
