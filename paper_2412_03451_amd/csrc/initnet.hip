// Learned plane initializer: kernels of the point-set network (gfx950).
//
// Forward: one 512-thread workgroup per 128 points of a view.  Layer 1
// (3 -> 256) runs on the vector ALU straight into an LDS tile of bfloat16
// activations; layers 2 and 3 (256 -> 256) are MFMA products
// (v_mfma_f32_32x32x16_bf16: each of the 8 waves owns a 64 x 64 block of
// the 128 x 256 output, A fragments from the LDS tile, B fragments from the
// transposed weights in L2); layer 2's output replaces layer 1's in LDS and
// layer 3's output never leaves registers: it is reduced to a per-column
// maximum (and the point attaining it) of the tile.  A second kernel takes
// the maximum over tiles and applies the head.  HBM traffic is the points
// (12 B each) and the per-tile maxima.
//
// Backward: only the point that attains a channel's maximum receives that
// channel's gradient, so the point layers are differentiated at B * 256 rows
// (one per (view, channel)).  Their activations are recomputed (no
// per-point state is stored by the forward), and the two 256-wide products
// (dW2 = h1^T dpre2 over the rows, dh1 = dpre2 W2^T) run on MFMA.  Every
// reduction over rows or views is taken in a fixed order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "initnet.h"
#include "planesplat.h"

extern "C" int ps_set_error(int code, const char* fmt, ...);

#define IN_HIP_CHECK(expr)                                                      \
  do {                                                                          \
    hipError_t _e = (expr);                                                     \
    if (_e != hipSuccess)                                                       \
      return ps_set_error(PS_ERR_HIP, "%s: %s", #expr, hipGetErrorString(_e));  \
  } while (0)

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int C = IN_C;
constexpr int TM = IN_TM;
constexpr int LDA = C + 8;    // LDS row of a tile, bfloat16 elements (16-byte pad)
constexpr float W_N = 0.25f;  // weight of the normal term of the set loss
constexpr float W_E = 0.25f;  // weight of the extent term
constexpr float R_MIN = 0.01f;

struct Offs {
  int64_t W1, b1, W2, b2, W3, b3, Wh, bh, n;
};
struct POffs {
  int64_t W1, W2t, W2, W3t, Wh, Wht, n;
};

__host__ __device__ inline Offs param_offs(int P) {
  Offs o;
  o.W1 = 0;
  o.b1 = o.W1 + 3 * C;
  o.W2 = o.b1 + C;
  o.b2 = o.W2 + (int64_t)C * C;
  o.W3 = o.b2 + C;
  o.b3 = o.W3 + (int64_t)C * C;
  o.Wh = o.b3 + C;
  o.bh = o.Wh + (int64_t)C * IN_OUT * P;
  o.n = o.bh + IN_OUT * P;
  return o;
}

__host__ __device__ inline POffs packed_offs(int P) {
  POffs o;
  o.W1 = 0;
  o.W2t = o.W1 + 3 * C;
  o.W2 = o.W2t + (int64_t)C * C;
  o.W3t = o.W2 + (int64_t)C * C;
  o.Wh = o.W3t + (int64_t)C * C;
  o.Wht = o.Wh + (int64_t)C * IN_OUT * P;
  o.n = o.Wht + (int64_t)C * IN_OUT * P;
  // keep every block 16-byte aligned: all sizes above are multiples of 8 elements
  return o;
}

// float -> bfloat16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t f2bf(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ f32x16 zero16() {
  f32x16 z;
#pragma unroll
  for (int i = 0; i < 16; ++i) z[i] = 0.f;
  return z;
}

__device__ __forceinline__ bf16x8 ld8(const uint16_t* p) { return *reinterpret_cast<const bf16x8*>(p); }

__device__ __forceinline__ f32x16 mfma(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// Accumulator element i of lane l of a 32 x 32 MFMA block: row and column.
__device__ __forceinline__ int acc_row(int i, int l) { return 8 * (i >> 2) + 4 * (l >> 5) + (i & 3); }
__device__ __forceinline__ int acc_col(int l) { return l & 31; }

// 128 x 32 block (every row of the tile, weight columns c0 .. c0+31) of
// H[r, :] . Wt[c, :] over K = 256: H is the LDS tile, Wt the transposed
// weights in global memory.  One B fragment per step feeds four MFMAs.
__device__ __forceinline__ void gemm_tile(const uint16_t* H, const uint16_t* __restrict__ Wt, int c0,
                                          f32x16 (&acc)[4]) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i] = zero16();
  const uint16_t* bp = Wt + (size_t)(c0 + (l & 31)) * C + 8 * (l >> 5);
  const uint16_t* ap = H + (l & 31) * LDA + 8 * (l >> 5);
#pragma unroll 4
  for (int k0 = 0; k0 < C; k0 += 16) {
    const bf16x8 b = ld8(bp + k0);
    const bf16x8 a0 = ld8(ap + k0), a1 = ld8(ap + 32 * LDA + k0);
    const bf16x8 a2 = ld8(ap + 64 * LDA + k0), a3 = ld8(ap + 96 * LDA + k0);
    acc[0] = mfma(a0, b, acc[0]);
    acc[1] = mfma(a1, b, acc[1]);
    acc[2] = mfma(a2, b, acc[2]);
    acc[3] = mfma(a3, b, acc[3]);
  }
}

// ---------------------------------------------------------------- forward
struct FwdArgs {
  const float* X;
  const float* master;
  const uint16_t* packed;
  int B, N, ntile;
  Offs o;
  POffs po;
  float* pv;      // [B][ntile][C] tile maxima
  int32_t* pi;    // [B][ntile][C] point attaining them
  uint16_t* dump; // [3][B*N][C] or null
};

template <bool DUMP>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4, 8))) void fwd_kernel(FwdArgs a) {
  __shared__ __attribute__((aligned(16))) uint16_t H[TM * LDA];
  const int tile = blockIdx.x, b = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int p0 = tile * TM;
  const size_t row0 = (size_t)b * a.N + p0;   // first point of the tile in [B*N]
  const float* X = a.X + row0 * 3;
  const uint16_t* W1 = a.packed + a.po.W1;
  const float* b1 = a.master + a.o.b1;
  const size_t BN = (size_t)a.B * a.N;
  // layer 1 on the vector ALU: thread = (column, half of the rows), the
  // column's weights in registers, the tile's points staged in LDS
  __shared__ float xs[TM * 3];
  for (int e = tid; e < TM * 3; e += 512) xs[e] = X[e];
  __syncthreads();
  {
    const int j = tid & (C - 1), half = tid >> 8;
    const float w0 = bf2f(W1[j]), w1 = bf2f(W1[C + j]), w2 = bf2f(W1[2 * C + j]), bj = b1[j];
    for (int m = half; m < TM; m += 2) {
      float v = fmaf(xs[3 * m], w0, bj);
      v = fmaf(xs[3 * m + 1], w1, v);
      v = fmaf(xs[3 * m + 2], w2, v);
      const uint16_t h = f2bf(fmaxf(v, 0.f));
      H[m * LDA + j] = h;
      if (DUMP) a.dump[(row0 + m) * C + j] = h;
    }
  }
  __syncthreads();
  const int c0 = w * 32;   // this wave's 32 output columns, every row
  const int col = c0 + acc_col(lane);
  f32x16 acc[4];
  // layer 2
  gemm_tile(H, a.packed + a.po.W2t, c0, acc);
  __syncthreads();   // every wave has read layer 1
  {
    const float bias = a.master[a.o.b2 + col];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = 32 * i + acc_row(v, lane);
        const uint16_t h = f2bf(fmaxf(acc[i][v] + bias, 0.f));
        H[row * LDA + col] = h;
        if (DUMP) a.dump[BN * C + (row0 + row) * C + col] = h;
      }
  }
  __syncthreads();
  // layer 3 and the tile's column maxima (all rows of a column are in this wave)
  gemm_tile(H, a.packed + a.po.W3t, c0, acc);
  const float bias = a.master[a.o.b3 + col];
  float best = -1.f;
  int bi = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int row = 32 * i + acc_row(v, lane);   // increasing along (i, v)
      const uint16_t hb = f2bf(fmaxf(acc[i][v] + bias, 0.f));
      const float h = bf2f(hb);
      if (DUMP) a.dump[2 * BN * C + (row0 + row) * C + col] = hb;
      if (h > best) {
        best = h;
        bi = row;
      }
    }
  const float ob = __shfl_xor(best, 32, 64);
  const int oi = __shfl_xor(bi, 32, 64);
  if (ob > best || (ob == best && oi < bi)) {
    best = ob;
    bi = oi;
  }
  if (lane < 32) {
    const size_t o = ((size_t)b * a.ntile + tile) * C + col;
    a.pv[o] = best;
    a.pi[o] = p0 + bi;
  }
}

struct HeadArgs {
  const float* master;
  const uint16_t* packed;
  int B, P12, ntile;
  Offs o;
  POffs po;
  const float* pv;
  const int32_t* pi;
  float* g;
  int32_t* arg;
  float* out;
};

// Maximum over the tiles (the earlier tile wins ties: smaller point index),
// then out = g Wh + bh.  One workgroup per (view, block of 256 outputs):
// each recomputes its view's maximum (32 KB of tile maxima at 4096 points)
// and the first block of the view stores it; a thread forms one output,
// the 256 terms in order.
__global__ __launch_bounds__(256) void head_kernel(HeadArgs a) {
  __shared__ float gs[C];
  const int b = blockIdx.x, c = threadIdx.x;
  float best = -1.f;
  int bi = 0;
  for (int t = 0; t < a.ntile; ++t) {
    const size_t o = ((size_t)b * a.ntile + t) * C + c;
    const float v = a.pv[o];
    if (v > best) {
      best = v;
      bi = a.pi[o];
    }
  }
  if (blockIdx.y == 0) {
    a.g[b * C + c] = best;
    a.arg[b * C + c] = bi;
  }
  gs[c] = best;
  __syncthreads();
  const int j = blockIdx.y * 256 + c;
  if (j >= a.P12) return;
  const uint16_t* Wh = a.packed + a.po.Wh + j;
  float acc = a.master[a.o.bh + j];
#pragma unroll 8
  for (int k = 0; k < C; ++k) acc = fmaf(gs[k], bf2f(Wh[(size_t)k * a.P12]), acc);
  a.out[(size_t)b * a.P12 + j] = acc;
}

// ---------------------------------------------------------------- set loss
struct LossArgs {
  const float* out;
  int B, P;
  const float* tgt;
  const int32_t* tgt_off;
  float* loss;
  float* d_out;
};

// rotation columns: plane normal n = third column of R(q) (Eq. 2-3)
__device__ inline void quat_normal(const float q[4], float n[3]) {
  const float w = q[0], x = q[1], y = q[2], z = q[3];
  n[0] = 2.f * (x * z + w * y);
  n[1] = 2.f * (y * z - w * x);
  n[2] = 1.f - 2.f * (x * x + y * y);
}

__device__ inline float softplus_f(float x) { return x > 20.f ? x : log1pf(expf(x)); }
__device__ inline float sigmoid_f(float x) { return 1.f / (1.f + expf(-x)); }

__device__ inline void target_desc(const float* t, float d[8]) {
  // center, unit normal, half-extents a >= b
  float q[4] = {t[3], t[4], t[5], t[6]};
  const float qn = sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int k = 0; k < 4; ++k) q[k] /= qn;
  float n[3];
  quat_normal(q, n);
  const float ex = 0.5f * (t[7] + t[8]), ey = 0.5f * (t[9] + t[10]);
  d[0] = t[0]; d[1] = t[1]; d[2] = t[2];
  d[3] = n[0]; d[4] = n[1]; d[5] = n[2];
  d[6] = fmaxf(ex, ey);
  d[7] = fminf(ex, ey);
}

constexpr int kTgtChunk = 256;

__global__ __launch_bounds__(256) void set_loss_kernel(LossArgs a) {
  __shared__ float td[kTgtChunk][8];
  __shared__ float wv[4];
  __shared__ int wi[4];
  __shared__ float red[4];
  const int b = blockIdx.x, p = threadIdx.x, lane = p & 63, wid = p >> 6;
  const bool act = p < a.P;
  const int P12 = IN_OUT * a.P;
  // decode proposal p
  float o[IN_OUT];
  for (int k = 0; k < IN_OUT; ++k) o[k] = act ? a.out[(size_t)b * P12 + IN_OUT * p + k] : 0.f;
  float qr[4] = {o[3] + 1.f, o[4], o[5], o[6]};
  const float qn = sqrtf(qr[0] * qr[0] + qr[1] * qr[1] + qr[2] * qr[2] + qr[3] * qr[3]);
  float q[4];
  for (int k = 0; k < 4; ++k) q[k] = qr[k] / qn;
  float rr[4];
  for (int k = 0; k < 4; ++k) rr[k] = softplus_f(o[7 + k]) + R_MIN;
  float n[3];
  quat_normal(q, n);
  const float ex = 0.5f * (rr[0] + rr[1]), ey = 0.5f * (rr[2] + rr[3]);
  const float ea = fmaxf(ex, ey), eb = fminf(ex, ey);
  // gradient accumulators of this proposal's geometric term
  float gc[3] = {0.f, 0.f, 0.f}, gn[3] = {0.f, 0.f, 0.f}, ga = 0.f, gb = 0.f;
  float geo = 0.f;
  bool matched = false;
  const int t0 = a.tgt_off[b], T = a.tgt_off[b + 1] - t0;
  for (int base = 0; base < T; base += kTgtChunk) {
    const int nt = min(kTgtChunk, T - base);
    __syncthreads();
    if (p < nt) {
      float d[8];
      target_desc(a.tgt + (size_t)(t0 + base + p) * 11, d);
      for (int k = 0; k < 8; ++k) td[p][k] = d[k];
    }
    __syncthreads();
    for (int t = 0; t < nt; ++t) {
      const float dc0 = o[0] - td[t][0], dc1 = o[1] - td[t][1], dc2 = o[2] - td[t][2];
      const float dot = n[0] * td[t][3] + n[1] * td[t][4] + n[2] * td[t][5];
      const float da = ea - td[t][6], db = eb - td[t][7];
      const float d = act ? (dc0 * dc0 + dc1 * dc1 + dc2 * dc2) + W_N * (1.f - dot * dot) + W_E * (da * da + db * db)
                          : INFINITY;
      // nearest proposal (smallest index on ties)
      float bv = d;
      int bi = p;
#pragma unroll
      for (int s = 32; s >= 1; s >>= 1) {
        const float ov = __shfl_xor(bv, s, 64);
        const int oi = __shfl_xor(bi, s, 64);
        if (ov < bv || (ov == bv && oi < bi)) {
          bv = ov;
          bi = oi;
        }
      }
      if (lane == 0) {
        wv[wid] = bv;
        wi[wid] = bi;
      }
      __syncthreads();
      float best = wv[0];
      int besti = wi[0];
      for (int k = 1; k < 4; ++k)
        if (wv[k] < best) {   // later waves hold larger indices
          best = wv[k];
          besti = wi[k];
        }
      __syncthreads();
      if (p == besti) {
        matched = true;
        geo += d;
        gc[0] += 2.f * dc0; gc[1] += 2.f * dc1; gc[2] += 2.f * dc2;
        const float s = -2.f * W_N * dot;
        gn[0] += s * td[t][3]; gn[1] += s * td[t][4]; gn[2] += s * td[t][5];
        ga += 2.f * W_E * da;
        gb += 2.f * W_E * db;
      }
    }
  }
  // loss of the view: mean over targets of the nearest distance + mean BCE
  const float y = matched ? 1.f : 0.f;
  const float bce = act ? softplus_f(o[11]) - y * o[11] : 0.f;
  const float invT = T > 0 ? 1.f / (float)T : 0.f;
  float part = geo * invT + bce / (float)a.P;
  for (int s = 32; s >= 1; s >>= 1) part += __shfl_xor(part, s, 64);
  if (lane == 0) red[wid] = part;
  __syncthreads();
  if (p == 0) a.loss[b] = ((red[0] + red[1]) + red[2]) + red[3];
  if (!act) return;
  // gradient of mean_b L_b
  const float sc = 1.f / (float)a.B;
  const float kg = invT * sc;
  float g[IN_OUT];
  g[0] = gc[0] * kg; g[1] = gc[1] * kg; g[2] = gc[2] * kg;
  g[11] = (sigmoid_f(o[11]) - y) / (float)a.P * sc;
  // half-extents: a = max(ex, ey), b = min(ex, ey); equal values share the gradient
  const float Ga = ga * kg, Gb = gb * kg;
  float gex, gey;
  if (ex > ey) {
    gex = Ga; gey = Gb;
  } else if (ex < ey) {
    gex = Gb; gey = Ga;
  } else {
    gex = 0.5f * (Ga + Gb); gey = gex;
  }
  const float grr[4] = {0.5f * gex, 0.5f * gex, 0.5f * gey, 0.5f * gey};
  for (int k = 0; k < 4; ++k) g[7 + k] = grr[k] * (o[7 + k] > 20.f ? 1.f : sigmoid_f(o[7 + k]));
  // normal -> unit quaternion (w, x, y, z) -> raw quaternion
  const float Gn0 = gn[0] * kg, Gn1 = gn[1] * kg, Gn2 = gn[2] * kg;
  const float w = q[0], x = q[1], yq = q[2], z = q[3];
  float gq[4];
  gq[0] = Gn0 * 2.f * yq - Gn1 * 2.f * x;
  gq[1] = Gn0 * 2.f * z - Gn1 * 2.f * w - Gn2 * 4.f * x;
  gq[2] = Gn0 * 2.f * w + Gn1 * 2.f * z - Gn2 * 4.f * yq;
  gq[3] = Gn0 * 2.f * x + Gn1 * 2.f * yq;
  const float qg = q[0] * gq[0] + q[1] * gq[1] + q[2] * gq[2] + q[3] * gq[3];
  for (int k = 0; k < 4; ++k) g[3 + k] = (gq[k] - q[k] * qg) / qn;
  for (int k = 0; k < IN_OUT; ++k) a.d_out[(size_t)b * P12 + IN_OUT * p + k] = g[k];
}

// ---------------------------------------------------------------- backward
struct BwdArgs {
  const float* master;
  const uint16_t* packed;
  int B, N, P12, R;
  int nzh;            // blocks of 256 head outputs (parts of dL/dg)
  Offs o;
  POffs po;
  const float* X;
  const float* g;
  const int32_t* arg;
  const float* d_out;
  float* grad;
  // workspace
  float* dg;          // [B][nzh][C]  parts of dL/dg
  uint16_t* h1T;      // [C][R]
  uint16_t* h1r;      // [R][C]
  uint16_t* dp2;      // [R][C]  dL/dpre2, bfloat16
  uint16_t* dp2T;     // [C][R]
  float* dp2f;        // [R][C]  dL/dpre2, float32
  uint16_t* h2r;      // [R][C]
  float* dp3;         // [R]
  float* dh1;         // [R][C]
  float* pw2;         // [parts][C][C] split-K partials of dW2
  float* colp;        // [R / kColChunk][5][C]
};

// dg[b][c] = sum_j Wh[c][j] d_out[b][j], in parts: workgroup (b, z) sums
// the head outputs j of block z (256 of them, in order) into
// dgp[b][z][c]; rows_kernel adds the parts in order.
__global__ __launch_bounds__(256) void head_dg_kernel(BwdArgs a) {
  const int b = blockIdx.x, z = blockIdx.y, c = threadIdx.x;
  const uint16_t* Wht = a.packed + a.po.Wht;
  const float* d = a.d_out + (size_t)b * a.P12;
  const int j1 = min(a.P12, 256 * z + 256);
  float acc = 0.f;
#pragma unroll 8
  for (int j = 256 * z; j < j1; ++j) acc = fmaf(bf2f(Wht[(size_t)j * C + c]), d[j], acc);
  a.dg[((size_t)b * a.nzh + z) * C + c] = acc;
}

// dWh[c][j] = sum_b g[b][c] d_out[b][j] (c < C) and dbh[j] = sum_b d_out[b][j]
// (c = C): one thread per output, the views in order.
__global__ __launch_bounds__(256) void head_dw_kernel(BwdArgs a) {
  const int64_t w = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t n_out = (int64_t)(C + 1) * a.P12;
  if (w >= n_out) return;
  const int c = (int)(w / a.P12), j = (int)(w % a.P12);
  float acc = 0.f;
  for (int b = 0; b < a.B; ++b) {
    const float d = a.d_out[(size_t)b * a.P12 + j];
    acc = c < C ? fmaf(a.g[b * C + c], d, acc) : acc + d;
  }
  if (c < C) a.grad[a.o.Wh + (size_t)c * a.P12 + j] = acc;
  else a.grad[a.o.bh + j] = acc;
}

// Rows r = b * C + c (the point attaining channel c of view b): recompute h1,
// pre2 / h2 and pre3[r][c]; form dL/dpre3 (channel c only), dL/dpre2.
__global__ __launch_bounds__(512) void rows_kernel(BwdArgs a) {
  __shared__ __attribute__((aligned(16))) uint16_t H[TM * LDA];
  __shared__ float d3[TM];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int rb = blockIdx.x * TM;   // first row of the block
  const uint16_t* W1 = a.packed + a.po.W1;
  const float* b1 = a.master + a.o.b1;
  for (int e = tid; e < TM * C; e += 512) {
    const int m = e % TM, j = e / TM;   // m fastest: coalesced transposed store
    const int r = rb + m;
    const int bv = r / C, ch = r % C;
    const int pt = a.arg[bv * C + ch];
    const float* x = a.X + ((size_t)bv * a.N + pt) * 3;
    float v = fmaf(x[0], bf2f(W1[j]), b1[j]);
    v = fmaf(x[1], bf2f(W1[C + j]), v);
    v = fmaf(x[2], bf2f(W1[2 * C + j]), v);
    const uint16_t h = f2bf(fmaxf(v, 0.f));
    H[m * LDA + j] = h;
    a.h1T[(size_t)j * a.R + r] = h;
  }
  __syncthreads();
  for (int e = tid; e < TM * C; e += 512) {   // row layout too (coalesced)
    const int m = e / C, j = e % C;
    a.h1r[(size_t)(rb + m) * C + j] = H[m * LDA + j];
  }
  __syncthreads();
  const int c0 = w * 32, col = c0 + acc_col(lane);
  f32x16 acc[4];
  gemm_tile(H, a.packed + a.po.W2t, c0, acc);
  __syncthreads();
  {
    const float bias = a.master[a.o.b2 + col];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = 32 * i + acc_row(v, lane);
        const uint16_t h = f2bf(fmaxf(acc[i][v] + bias, 0.f));
        H[row * LDA + col] = h;
        a.h2r[(size_t)(rb + row) * C + col] = h;
      }
  }
  __syncthreads();
  // pre3[r][c_r] = h2[r] . W3[:, c_r] + b3[c_r]: four threads per row
  {
    const int m = tid >> 2, part = tid & 3;
    const int r = rb + m, ch = r % C;
    const uint16_t* w3 = a.packed + a.po.W3t + (size_t)ch * C;   // row ch of W3^T = column ch of W3
    float s = 0.f;
    for (int k = part * 64; k < part * 64 + 64; ++k) s = fmaf(bf2f(H[m * LDA + k]), bf2f(w3[k]), s);
    s += __shfl_xor(s, 1, 64);
    s += __shfl_xor(s, 2, 64);
    if (part == 0) {
      const float pre3 = s + a.master[a.o.b3 + ch];
      float dgr = 0.f;   // dL/dg of (view, channel): its parts in order
      for (int z = 0; z < a.nzh; ++z) dgr += a.dg[((size_t)(r / C) * a.nzh + z) * C + ch];
      const float d = pre3 > 0.f ? dgr : 0.f;
      d3[m] = d;
      a.dp3[r] = d;
    }
  }
  __syncthreads();
  // dL/dpre2[r][k] = dL/dpre3[r] W3[k][c_r] [pre2 > 0]
  for (int e = tid; e < TM * C; e += 512) {
    const int m = e / C, k = e % C;
    const int r = rb + m, ch = r % C;
    const float h2 = bf2f(H[m * LDA + k]);
    const float d = h2 > 0.f ? d3[m] * bf2f(a.packed[a.po.W3t + (size_t)ch * C + k]) : 0.f;
    a.dp2f[(size_t)r * C + k] = d;
    const uint16_t db = f2bf(d);
    a.dp2[(size_t)r * C + k] = db;
  }
  for (int e = tid; e < TM * C; e += 512) {   // the same values, transposed (coalesced)
    const int m = e % TM, k = e / TM;
    const int r = rb + m, ch = r % C;
    const float h2 = bf2f(H[m * LDA + k]);
    const float d = h2 > 0.f ? d3[m] * bf2f(a.packed[a.po.W3t + (size_t)ch * C + k]) : 0.f;
    a.dp2T[(size_t)k * a.R + r] = f2bf(d);
  }
}

// Cm[z][m][n] = sum_{k in chunk z} A[m][k] Bt[n][k]  (bfloat16 operands,
// float32 accumulation); 128 x 128 per workgroup, 64 x 64 per wave.
struct GemmArgs {
  const uint16_t* A;
  int64_t lda;
  const uint16_t* Bt;
  int64_t ldb;
  float* Cm;
  int64_t ldc;
  int K, kc;
  int64_t zstride;
};

__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int m0 = blockIdx.y * 128 + (w >> 1) * 64, n0 = blockIdx.x * 128 + (w & 1) * 64;
  const int kb = blockIdx.z * g.kc, ke = min(g.K, kb + g.kc);
  f32x16 acc[2][2] = {{zero16(), zero16()}, {zero16(), zero16()}};
  const uint16_t* ap0 = g.A + (size_t)(m0 + (l & 31)) * g.lda + 8 * (l >> 5);
  const uint16_t* ap1 = ap0 + 32 * g.lda;
  const uint16_t* bp0 = g.Bt + (size_t)(n0 + (l & 31)) * g.ldb + 8 * (l >> 5);
  const uint16_t* bp1 = bp0 + 32 * g.ldb;
#pragma unroll 4
  for (int k0 = kb; k0 < ke; k0 += 16) {
    const bf16x8 a0 = ld8(ap0 + k0), a1 = ld8(ap1 + k0);
    const bf16x8 b0 = ld8(bp0 + k0), b1 = ld8(bp1 + k0);
    acc[0][0] = mfma(a0, b0, acc[0][0]);
    acc[0][1] = mfma(a0, b1, acc[0][1]);
    acc[1][0] = mfma(a1, b0, acc[1][0]);
    acc[1][1] = mfma(a1, b1, acc[1][1]);
  }
  float* Cz = g.Cm + blockIdx.z * g.zstride;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v)
        Cz[(size_t)(m0 + 32 * i + acc_row(v, l)) * g.ldc + n0 + 32 * j + acc_col(l)] = acc[i][j][v];
}

constexpr int kColChunk = 64;   // rows per column-sum chunk (enough chunks to fill the chip)

// Column sums over a chunk of rows (thread = column): dW1 (3), db1, db2.
__global__ __launch_bounds__(256) void colpart_kernel(BwdArgs a) {
  const int j = threadIdx.x, chunk = blockIdx.x;
  float s[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
  const int r0 = chunk * kColChunk, r1 = min(a.R, r0 + kColChunk);
  for (int r = r0; r < r1; ++r) {
    const int bv = r / C, ch = r % C;
    const float* x = a.X + ((size_t)bv * a.N + a.arg[bv * C + ch]) * 3;
    const float h1 = bf2f(a.h1r[(size_t)r * C + j]);
    const float d1 = h1 > 0.f ? a.dh1[(size_t)r * C + j] : 0.f;
    s[0] = fmaf(x[0], d1, s[0]);
    s[1] = fmaf(x[1], d1, s[1]);
    s[2] = fmaf(x[2], d1, s[2]);
    s[3] += d1;
    s[4] += a.dp2f[(size_t)r * C + j];
  }
  for (int k = 0; k < 5; ++k) a.colp[((size_t)chunk * 5 + k) * C + j] = s[k];
}

// dW1, db1, db2: one wave per (value, column), lanes over chunks.
__global__ __launch_bounds__(256) void colsum_kernel(BwdArgs a, int nchunk) {
  const int w = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (w >= 5 * C) return;
  const int k = w / C, j = w % C;
  float acc = 0.f;
  for (int ck = lane; ck < nchunk; ck += 64) acc += a.colp[((size_t)ck * 5 + k) * C + j];
  for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (lane == 0) {
    if (k < 3) a.grad[a.o.W1 + k * C + j] = acc;
    else if (k == 3) a.grad[a.o.b1 + j] = acc;
    else a.grad[a.o.b2 + j] = acc;
  }
}

// dW2 over the split-K parts; dW3, db3 over views.  Block = row of dW2 /
// column of dW3, thread = the other index.
__global__ __launch_bounds__(256) void wgrad_kernel(BwdArgs a, int nz) {
  const int row = blockIdx.x, t = threadIdx.x;
  float s = 0.f;
  for (int z = 0; z < nz; ++z) s += a.pw2[((size_t)z * C + row) * C + t];
  a.grad[a.o.W2 + (size_t)row * C + t] = s;
  float s3 = 0.f, sb = 0.f;
  for (int b = 0; b < a.B; ++b) {
    const int r = b * C + row;
    const float d = a.dp3[r];
    s3 = fmaf(bf2f(a.h2r[(size_t)r * C + t]), d, s3);
    sb += d;
  }
  a.grad[a.o.W3 + (size_t)t * C + row] = s3;
  if (t == 0) a.grad[a.o.b3 + row] = sb;
}

// ---------------------------------------------------------------- optimiser
__global__ void pack_kernel(const float* master, uint16_t* packed, int P, Offs o, POffs po) {
  const int64_t P12 = (int64_t)IN_OUT * P;
  const int64_t n = 3 * C + 3 * (int64_t)C * C + 2 * (int64_t)C * P12;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = e;
    if (i < 3 * C) { packed[po.W1 + i] = f2bf(master[o.W1 + i]); continue; }
    i -= 3 * C;
    if (i < (int64_t)C * C) {   // W2t[o][i] = W2[i][o]
      const int64_t r = i / C, c = i % C;
      packed[po.W2t + i] = f2bf(master[o.W2 + c * C + r]);
      continue;
    }
    i -= (int64_t)C * C;
    if (i < (int64_t)C * C) { packed[po.W2 + i] = f2bf(master[o.W2 + i]); continue; }
    i -= (int64_t)C * C;
    if (i < (int64_t)C * C) {
      const int64_t r = i / C, c = i % C;
      packed[po.W3t + i] = f2bf(master[o.W3 + c * C + r]);
      continue;
    }
    i -= (int64_t)C * C;
    if (i < C * P12) { packed[po.Wh + i] = f2bf(master[o.Wh + i]); continue; }
    i -= C * P12;
    {   // Wht[j][c] = Wh[c][j]
      const int64_t j = i / C, c = i % C;
      packed[po.Wht + i] = f2bf(master[o.Wh + c * P12 + j]);
    }
  }
}

__global__ void adam_kernel(float* th, float* m, float* v, const float* g, int64_t n, const int32_t* step, float lr,
                            float b1, float b2, float eps) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int s = *step;
  const float bc1 = 1.f - powf(b1, (float)s), bc2 = 1.f - powf(b2, (float)s);
  const float gi = g[i];
  const float mi = fmaf(b1, m[i], (1.f - b1) * gi);
  const float vi = fmaf(b2, v[i], (1.f - b2) * gi * gi);
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

inline int64_t ws_align(int64_t floats) { return (floats + 63) & ~int64_t(63); }

// split-K parts of the dW2 product: enough workgroups to fill the chip,
// each over a multiple of 16 rows
inline int wgrad_parts(int64_t R) {
  int nz = 1;
  while (nz < 64 && R / (2 * nz) >= 512 && (R / (2 * nz)) % 16 == 0 && R % (2 * nz) == 0) nz *= 2;
  return nz;
}

struct BwdWs {
  int64_t dg, h1T, h1r, dp2, dp2T, dp2f, h2r, dp3, dh1, pw2, colp, n;
};
inline BwdWs bwd_ws(int B, int P) {
  const int64_t R = (int64_t)B * C;
  BwdWs w;
  int64_t o = 0;
  w.dg = o; o += ws_align(R * ((IN_OUT * P + 255) / 256));
  w.h1T = o; o += ws_align(R * C / 2);
  w.h1r = o; o += ws_align(R * C / 2);
  w.dp2 = o; o += ws_align(R * C / 2);
  w.dp2T = o; o += ws_align(R * C / 2);
  w.dp2f = o; o += ws_align(R * C);
  w.h2r = o; o += ws_align(R * C / 2);
  w.dp3 = o; o += ws_align(R);
  w.dh1 = o; o += ws_align(R * C);
  w.pw2 = o; o += ws_align((int64_t)wgrad_parts(R) * C * C);
  w.colp = o; o += ws_align(((R + kColChunk - 1) / kColChunk) * 5 * (int64_t)C);
  w.n = o;
  return w;
}

}  // namespace

extern "C" int64_t initnet_param_count(int P) { return P < 1 || P > IN_PMAX ? 0 : param_offs(P).n; }
extern "C" int64_t initnet_packed_count(int P) { return P < 1 || P > IN_PMAX ? 0 : packed_offs(P).n; }
extern "C" int64_t initnet_forward_ws(int B, int N) {
  if (B < 1 || N < TM || N % TM) return 0;
  return 2 * ws_align((int64_t)B * (N / TM) * C);
}
extern "C" int64_t initnet_backward_ws(int B, int P) {
  if (B < 2 || B % 2 || P < 1 || P > IN_PMAX) return 0;
  return bwd_ws(B, P).n;
}

static int check_p(int P, const char* who) {
  if (P < 1 || P > IN_PMAX) return ps_set_error(PS_ERR_INVALID, "%s: P=%d not in 1..%d", who, P, IN_PMAX);
  return PS_OK;
}

extern "C" int initnet_pack(const float* master, int P, uint16_t* packed, void* stream) {
  if (int rc = check_p(P, "initnet_pack")) return rc;
  if (!master || !packed) return ps_set_error(PS_ERR_INVALID, "initnet_pack: null pointer");
  hipLaunchKernelGGL(pack_kernel, dim3(1024), dim3(256), 0, (hipStream_t)stream, master, packed, P, param_offs(P),
                     packed_offs(P));
  IN_HIP_CHECK(hipGetLastError());
  return PS_OK;
}

extern "C" int initnet_forward(const float* master, const uint16_t* packed, int P, const float* X, int B, int N,
                               float* g, int32_t* arg, float* out, float* ws, uint16_t* dump, void* stream) {
  if (int rc = check_p(P, "initnet_forward")) return rc;
  if (!master || !packed || !X || !g || !arg || !out || !ws)
    return ps_set_error(PS_ERR_INVALID, "initnet_forward: null pointer");
  if (B < 1 || N < TM || N % TM) return ps_set_error(PS_ERR_INVALID, "initnet_forward: B=%d N=%d (N a multiple of %d)", B, N, TM);
  if (((uintptr_t)ws) & 255) return ps_set_error(PS_ERR_INVALID, "initnet_forward: workspace not 256-byte aligned");
  hipStream_t st = (hipStream_t)stream;
  FwdArgs a;
  a.X = X; a.master = master; a.packed = packed;
  a.B = B; a.N = N; a.ntile = N / TM;
  a.o = param_offs(P); a.po = packed_offs(P);
  const int64_t half = ws_align((int64_t)B * a.ntile * C);
  a.pv = ws;
  a.pi = (int32_t*)(ws + half);
  a.dump = dump;
  if (dump)
    hipLaunchKernelGGL(fwd_kernel<true>, dim3(a.ntile, B), dim3(512), 0, st, a);
  else
    hipLaunchKernelGGL(fwd_kernel<false>, dim3(a.ntile, B), dim3(512), 0, st, a);
  HeadArgs h;
  h.master = master; h.packed = packed; h.B = B; h.P12 = IN_OUT * P; h.ntile = a.ntile;
  h.o = a.o; h.po = a.po; h.pv = a.pv; h.pi = a.pi; h.g = g; h.arg = arg; h.out = out;
  hipLaunchKernelGGL(head_kernel, dim3(B, (h.P12 + 255) / 256), dim3(256), 0, st, h);
  IN_HIP_CHECK(hipGetLastError());
  return PS_OK;
}

extern "C" int initnet_set_loss(const float* out, int B, int P, const float* tgt, const int32_t* tgt_off, float* loss,
                                float* d_out, void* stream) {
  if (int rc = check_p(P, "initnet_set_loss")) return rc;
  if (!out || !tgt_off || !loss || !d_out) return ps_set_error(PS_ERR_INVALID, "initnet_set_loss: null pointer");
  if (B < 1) return ps_set_error(PS_ERR_INVALID, "initnet_set_loss: B=%d", B);
  LossArgs a{out, B, P, tgt, tgt_off, loss, d_out};
  hipLaunchKernelGGL(set_loss_kernel, dim3(B), dim3(256), 0, (hipStream_t)stream, a);
  IN_HIP_CHECK(hipGetLastError());
  return PS_OK;
}

extern "C" int initnet_backward(const float* master, const uint16_t* packed, int P, const float* X, int B, int N,
                                const float* g, const int32_t* arg, const float* d_out, float* grad, float* ws,
                                void* stream) {
  if (int rc = check_p(P, "initnet_backward")) return rc;
  if (!master || !packed || !X || !g || !arg || !d_out || !grad || !ws)
    return ps_set_error(PS_ERR_INVALID, "initnet_backward: null pointer");
  if (B < 2 || B % 2 || N < 1) return ps_set_error(PS_ERR_INVALID, "initnet_backward: B=%d must be even and >= 2", B);
  if (((uintptr_t)ws) & 255) return ps_set_error(PS_ERR_INVALID, "initnet_backward: workspace not 256-byte aligned");
  hipStream_t st = (hipStream_t)stream;
  const BwdWs w = bwd_ws(B, P);
  BwdArgs a;
  a.master = master; a.packed = packed; a.B = B; a.N = N; a.P12 = IN_OUT * P; a.R = B * C;
  a.nzh = (a.P12 + 255) / 256;
  a.o = param_offs(P); a.po = packed_offs(P);
  a.X = X; a.g = g; a.arg = arg; a.d_out = d_out; a.grad = grad;
  a.dg = ws + w.dg;
  a.h1T = (uint16_t*)(ws + w.h1T);
  a.h1r = (uint16_t*)(ws + w.h1r);
  a.dp2 = (uint16_t*)(ws + w.dp2);
  a.dp2T = (uint16_t*)(ws + w.dp2T);
  a.dp2f = ws + w.dp2f;
  a.h2r = (uint16_t*)(ws + w.h2r);
  a.dp3 = ws + w.dp3;
  a.dh1 = ws + w.dh1;
  a.pw2 = ws + w.pw2;
  a.colp = ws + w.colp;
  const int R = a.R;
  hipLaunchKernelGGL(head_dg_kernel, dim3(B, a.nzh), dim3(256), 0, st, a);
  hipLaunchKernelGGL(head_dw_kernel, dim3((unsigned)(((int64_t)(C + 1) * a.P12 + 255) / 256)), dim3(256), 0, st, a);
  hipLaunchKernelGGL(rows_kernel, dim3(R / TM), dim3(512), 0, st, a);
  // dW2 partials: [k1][k2] = sum_r h1T[k1][r] dp2T[k2][r], split over row chunks
  const int nz = wgrad_parts(R);
  GemmArgs g2{a.h1T, R, a.dp2T, R, a.pw2, C, R, R / nz, (int64_t)C * C};
  hipLaunchKernelGGL(gemm_kernel, dim3(C / 128, C / 128, nz), dim3(256), 0, st, g2);
  // dh1[r][k1] = sum_k2 dp2[r][k2] W2[k1][k2]
  GemmArgs g1{a.dp2, C, packed + a.po.W2, C, a.dh1, C, C, C, 0};
  hipLaunchKernelGGL(gemm_kernel, dim3(C / 128, R / 128, 1), dim3(256), 0, st, g1);
  const int nchunk = (R + kColChunk - 1) / kColChunk;
  hipLaunchKernelGGL(colpart_kernel, dim3(nchunk), dim3(256), 0, st, a);
  hipLaunchKernelGGL(colsum_kernel, dim3(5 * C / 4), dim3(256), 0, st, a, nchunk);
  hipLaunchKernelGGL(wgrad_kernel, dim3(C), dim3(256), 0, st, a, nz);
  IN_HIP_CHECK(hipGetLastError());
  return PS_OK;
}

extern "C" int initnet_adam(float* master, float* m, float* v, const float* grad, int64_t n, const int32_t* step,
                            float lr, float beta1, float beta2, float eps, void* stream) {
  if (!master || !m || !v || !grad || !step || n < 0) return ps_set_error(PS_ERR_INVALID, "initnet_adam: bad argument");
  if (n == 0) return PS_OK;
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, master, m, v,
                     grad, n, step, lr, beta1, beta2, eps);
  IN_HIP_CHECK(hipGetLastError());
  return PS_OK;
}
