// plane_project: one thread per (plane, job) record.
//
// Builds the camera-frame record of Sec. 3.1 (Eq. 2-3) and the affine-in-pixel
// numerators / denominator of the ray-plane intersection (Eq. 4) and the
// in-plane coordinates (Eq. 6), plus the screen footprint outside which the
// splat weight is below tau.  w >= tau holds exactly when
// -(r^{x-} + delta) <= P_X <= r^{x+} + delta and likewise for P_Y, with the
// closed-form fringe margin delta(lambda); so the footprint is the rectangle
// grown by delta, clipped to z >= z_near and projected.
#include "ps_internal.h"

using namespace ps;

int ps_check_ws(const ps_layout* L, const void* ws, const char* who);

namespace {

struct ProjArgs {
  const ps_slot* slots;
  int S, R;
  const float* center;
  const float* quat;
  const float* radii;
  const ps_camera* cams;
  const float* lambda;
  int n_cams;
  float tau, z_near;
  double flog;   // filter_log(tau, mode)
  int mode, two_sided;
  Rec* recs;
  BinRec* brecs;
  int32_t* clear;   // the binning counts (record counts .. tile counts) to zero
  int64_t n_clear;
};

__device__ inline void store_culled(Rec* recs, BinRec* brecs, int r, int slot) {
  Rec z = {};
  z.cull = 1;
  z.px0 = 1; z.px1 = 0; z.py0 = 1; z.py1 = 0;
  recs[r] = z;
  BinRec b = {};
  b.nedge = 0;
  b.tx0 = 1; b.tx1 = 0; b.ty0 = 1; b.ty1 = 0;
  b.slot = slot;
  brecs[r] = b;
}

// affine (u, v) coefficients of c . d(u, v), d = ((u - cx)/fx, (v - cy)/fy, 1)
__device__ inline void affine(const double c[3], const ps_camera& cam, double& c0, double& cu, double& cv) {
  cu = c[0] / (double)cam.fx;
  cv = c[1] / (double)cam.fy;
  c0 = c[2] - cu * (double)cam.cx - cv * (double)cam.cy;
}

__global__ __launch_bounds__(64) void project_kernel(ProjArgs a) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  // the counts tile_bin accumulates start from zero (this saves the binning a
  // clearing launch of its own)
  if (r < a.n_clear) a.clear[r] = 0;
  if (r >= a.R) return;
  const int s = find_slot_by_rec(a.slots, a.S, r);
  const ps_slot sl = a.slots[s];
  const int k = sl.plane_begin + (r - sl.rec_begin);
  if (sl.cam < 0 || sl.cam >= a.n_cams) {
    store_culled(a.recs, a.brecs, r, s);
    return;
  }
  const ps_camera cam = a.cams[sl.cam];
  Frame f;
  if (!plane_frame(a.center, a.quat, k, cam, f) || f.h == 0.0) {
    store_culled(a.recs, a.brecs, r, s);
    return;
  }
  const double lam = (double)a.lambda[0];
  const double delta = fringe_margin(lam, a.flog, a.mode);
  const float rad[4] = {a.radii[4 * k + 0], a.radii[4 * k + 1], a.radii[4 * k + 2], a.radii[4 * k + 3]};

  Rec rec;
  double cx[3], cy[3];
  for (int i = 0; i < 3; ++i) {
    cx[i] = f.h * f.vxc[i] - f.pvx * f.nc[i];
    cy[i] = f.h * f.vyc[i] - f.pvy * f.nc[i];
  }
  affine(f.nc, cam, rec.D0, rec.Du, rec.Dv);
  affine(cx, cam, rec.X0, rec.Xu, rec.Xv);
  affine(cy, cam, rec.Y0, rec.Yu, rec.Yv);
  rec.h = f.h;
  rec.rxp = rad[0]; rec.rxm = rad[1]; rec.ryp = rad[2]; rec.rym = rad[3];
  // facing sign: every hit has sign(d.n) = sign(h), so the camera-facing
  // normal is -sign(h) R n (two-sided), constant over the job
  const double sgn = a.two_sided ? (f.h > 0.0 ? -1.0 : 1.0) : 1.0;
  rec.nx = (float)(sgn * f.nc[0]);
  rec.ny = (float)(sgn * f.nc[1]);
  rec.nz = (float)(sgn * f.nc[2]);
  rec.cull = 0;
  rec.pvx = (float)f.pvx;
  rec.pvy = (float)f.pvy;

  // grown rectangle corners in camera coordinates (x_c = R x + t)
  // (mode 2, the Gaussian: w >= tau inside the ellipse |P / r| <= sqrt(Q),
  // so the rectangle of the radii times sqrt(Q))
  const double ext = a.mode == 2 ? sqrt(delta) : 1.0, grow = a.mode == 2 ? 0.0 : delta;
  const double gx[2] = {(double)rad[0] * ext + grow, -((double)rad[1] * ext + grow)};
  const double gy[2] = {(double)rad[2] * ext + grow, -((double)rad[3] * ext + grow)};
  double corner[4][3];
  const double ab[4][2] = {{gx[0], gy[0]}, {gx[1], gy[0]}, {gx[1], gy[1]}, {gx[0], gy[1]}};
  for (int c = 0; c < 4; ++c) {
    double xw[3];
    for (int i = 0; i < 3; ++i) xw[i] = f.p[i] + ab[c][0] * f.vx[i] + ab[c][1] * f.vy[i];
    for (int i = 0; i < 3; ++i)
      corner[c][i] = (double)cam.R[3 * i] * xw[0] + (double)cam.R[3 * i + 1] * xw[1] +
                     (double)cam.R[3 * i + 2] * xw[2] + (double)cam.t[i];
  }
  // clip to z >= z_near (one plane of Sutherland-Hodgman).  Edge c of the
  // quad (corner c -> corner c+1) gives at most two vertices of the clipped
  // polygon, kept in fixed slots 2c (corner c, when inside) and 2c + 1 (the
  // crossing, when the edge crosses): the valid slots in slot order are the
  // polygon in order, and every array index below is a constant (no
  // scratch memory).
  const double zn = (double)a.z_near;
  double px[8], py[8], pz[8];
  bool ok[8];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double* A = corner[c];
    const double* B = corner[(c + 1) & 3];
    const bool ina = A[2] >= zn, inb = B[2] >= zn;
    ok[2 * c] = ina;
    px[2 * c] = A[0]; py[2 * c] = A[1]; pz[2 * c] = A[2];
    ok[2 * c + 1] = ina != inb;
    const double t = (ina != inb) ? (zn - A[2]) / (B[2] - A[2]) : 0.0;
    px[2 * c + 1] = A[0] + t * (B[0] - A[0]);
    py[2 * c + 1] = A[1] + t * (B[1] - A[1]);
    pz[2 * c + 1] = zn;
  }
  int np = 0;
#pragma unroll
  for (int c = 0; c < 8; ++c) np += ok[c] ? 1 : 0;
  if (np == 0) {
    store_culled(a.recs, a.brecs, r, s);
    return;
  }
  double zmin = 1e300, umin = 1e300, umax = -1e300, vmin = 1e300, vmax = -1e300;
  double pu[8], pv[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const double z = ok[c] ? pz[c] : 1.0;
    pu[c] = (double)cam.fx * px[c] / z + (double)cam.cx;
    pv[c] = (double)cam.fy * py[c] / z + (double)cam.cy;
    if (ok[c]) {
      zmin = fmin(zmin, pz[c]);
      umin = fmin(umin, pu[c]); umax = fmax(umax, pu[c]);
      vmin = fmin(vmin, pv[c]); vmax = fmax(vmax, pv[c]);
    }
  }
  // pixel i is inside when umin <= i + 1/2 <= umax; one pixel of guard
  const double W = sl.width, H = sl.height;
  const double i0 = fmax(0.0, floor(umin - 0.5) - 1.0), i1 = fmin(W - 1.0, ceil(umax - 0.5) + 1.0);
  const double j0 = fmax(0.0, floor(vmin - 0.5) - 1.0), j1 = fmin(H - 1.0, ceil(vmax - 0.5) + 1.0);
  if (!(i0 <= i1) || !(j0 <= j1)) {
    store_culled(a.recs, a.brecs, r, s);
    return;
  }
  rec.px0 = (int16_t)i0; rec.px1 = (int16_t)i1;
  rec.py0 = (int16_t)j0; rec.py1 = (int16_t)j1;
  a.recs[r] = rec;

  // next valid slot after each slot, cyclically (itself when it is the only one)
  int nxt[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    int n = c;
#pragma unroll
    for (int k = 7; k >= 1; --k)
      if (ok[(c + k) & 7]) n = (c + k) & 7;
    nxt[c] = n;
  }
  // orientation: signed area of the polygon, summed from its first vertex
  double area = 0.0;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    if (!ok[c]) continue;
    double un = pu[0], vn = pv[0];
#pragma unroll
    for (int d = 0; d < 8; ++d)
      if (d == nxt[c]) { un = pu[d]; vn = pv[d]; }
    area += pu[c] * vn - un * pv[c];
  }
  BinRec* bo = a.brecs + r;
  for (int e = 0; e < 5; ++e) bo->edge[e][0] = bo->edge[e][1] = bo->edge[e][2] = 0.0;
  if (np >= 3 && fabs(area) > 1e-3) {
    // signed distance to each edge, positive inside: edges run from each
    // vertex to the next (counter-clockwise polygon) or back (clockwise)
    bo->nedge = np;
    int e = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      if (!ok[c]) continue;
      double un = pu[0], vn = pv[0];
#pragma unroll
      for (int d = 0; d < 8; ++d)
        if (d == nxt[c]) { un = pu[d]; vn = pv[d]; }
      const double ua = area > 0 ? pu[c] : un, va = area > 0 ? pv[c] : vn;
      const double ub = area > 0 ? un : pu[c], vb = area > 0 ? vn : pv[c];
      const double ex = ub - ua, ey = vb - va;
      const double len = sqrt(ex * ex + ey * ey);
      if (len > 0.0) {
        bo->edge[e][0] = -ey / len;
        bo->edge[e][1] = ex / len;
        bo->edge[e][2] = (ey * ua - ex * va) / len;
      } else {  // repeated vertex: no constraint
        bo->edge[e][2] = 1.0;
      }
      ++e;
    }
  } else {
    bo->nedge = -1;
  }
  // depth lower bound over the grown, clipped rectangle, rounded down.  The
  // ray parameter of a hit equals its camera z only up to the float32
  // rounding of R (R R^T = I to ~1e-7): a relative margin of 4e-6 covers it.
  bo->tlb = __double2float_rd(fmax(zmin, zn) * (1.0 - 4e-6));
  bo->tx0 = (int)i0 / sl.tile_w; bo->tx1 = (int)i1 / sl.tile_w;
  bo->ty0 = (int)j0 / sl.tile_h; bo->ty1 = (int)j1 / sl.tile_h;
  bo->slot = s;
  bo->pad[0] = bo->pad[1] = bo->pad[2] = 0;
}

}  // namespace

extern "C" int plane_project(const ps_layout* L, void* ws, const float* center, const float* quat,
                             const float* radii, int K, const ps_camera* cams, int n_cams,
                             const float* lambda, const ps_params* prm, void* stream) {
  int rc = ps_check_ws(L, ws, "plane_project");
  if (rc) return rc;
  // an empty plane set (K = 0) may come with null plane arrays
  if (!cams || !lambda || !prm || K < 0 || (K > 0 && (!center || !quat || !radii)))
    return ps_set_error(PS_ERR_INVALID, "plane_project: null pointer or K < 0");
  if (K < L->n_planes) return ps_set_error(PS_ERR_INVALID, "plane_project: K=%d < planes referenced %d", K, L->n_planes);
  if (n_cams <= 0) return ps_set_error(PS_ERR_INVALID, "plane_project: n_cams <= 0");
  if (!(prm->tau > 0.f && prm->tau < 1.f) || !(prm->z_near > 0.f) || prm->M < 1 || prm->M > kMaxM ||
      (prm->weight_mode < 0 || prm->weight_mode > 2))
    return ps_set_error(PS_ERR_INVALID, "plane_project: bad ps_params");
  char* base = (char*)ws;
  ProjArgs a;
  // record counts, their offsets and the tile counts of tile_bin: adjacent
  // regions (the gaps between them are padding), cleared by the same launch
  static_assert(R_REC_OFF == R_REC_CNT + 1 && R_TILE_CNT == R_REC_OFF + 1, "region order");
  a.clear = (int32_t*)(base + L->region[R_REC_CNT]);
  a.n_clear = (int64_t)(L->region[R_TILE_CNT] - L->region[R_REC_CNT]) / 4 + L->n_tiles + 1;
  a.slots = (const ps_slot*)(base + L->region[R_SLOTS]);
  a.S = L->n_slots;
  a.R = L->n_records;
  a.center = center; a.quat = quat; a.radii = radii;
  a.cams = cams; a.lambda = lambda; a.n_cams = n_cams;
  a.tau = prm->tau; a.z_near = prm->z_near; a.mode = prm->weight_mode; a.two_sided = prm->two_sided;
  a.flog = filter_log((double)prm->tau, prm->weight_mode);
  a.recs = (Rec*)(base + L->region[R_REC]);
  a.brecs = (BinRec*)(base + L->region[R_BINREC]);
  const int64_t n = a.R > a.n_clear ? (int64_t)a.R : a.n_clear;
  hipLaunchKernelGGL(project_kernel, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, (hipStream_t)stream, a);
  PS_HIP_CHECK(hipGetLastError());
  return PS_OK;
}
