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
  int mode, two_sided;
  Rec* recs;
  BinRec* brecs;
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

__global__ __launch_bounds__(256) void project_kernel(ProjArgs a) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
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
  const double delta = fringe_margin(lam, (double)a.tau, a.mode);
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
  const double gx[2] = {(double)rad[0] + delta, -((double)rad[1] + delta)};
  const double gy[2] = {(double)rad[2] + delta, -((double)rad[3] + delta)};
  double corner[4][3];
  const double ab[4][2] = {{gx[0], gy[0]}, {gx[1], gy[0]}, {gx[1], gy[1]}, {gx[0], gy[1]}};
  for (int c = 0; c < 4; ++c) {
    double xw[3];
    for (int i = 0; i < 3; ++i) xw[i] = f.p[i] + ab[c][0] * f.vx[i] + ab[c][1] * f.vy[i];
    for (int i = 0; i < 3; ++i)
      corner[c][i] = (double)cam.R[3 * i] * xw[0] + (double)cam.R[3 * i + 1] * xw[1] +
                     (double)cam.R[3 * i + 2] * xw[2] + (double)cam.t[i];
  }
  // clip to z >= z_near (one plane of Sutherland-Hodgman)
  double poly[5][3];
  int np = 0;
  const double zn = (double)a.z_near;
  for (int c = 0; c < 4; ++c) {
    const double* A = corner[c];
    const double* B = corner[(c + 1) & 3];
    const bool ina = A[2] >= zn, inb = B[2] >= zn;
    if (ina) {
      for (int i = 0; i < 3; ++i) poly[np][i] = A[i];
      ++np;
    }
    if (ina != inb) {
      const double t = (zn - A[2]) / (B[2] - A[2]);
      for (int i = 0; i < 3; ++i) poly[np][i] = A[i] + t * (B[i] - A[i]);
      poly[np][2] = zn;
      ++np;
    }
  }
  if (np == 0) {
    store_culled(a.recs, a.brecs, r, s);
    return;
  }
  double zmin = poly[0][2], umin = 1e300, umax = -1e300, vmin = 1e300, vmax = -1e300;
  double pu[5], pv[5];
  for (int c = 0; c < np; ++c) {
    zmin = fmin(zmin, poly[c][2]);
    pu[c] = (double)cam.fx * poly[c][0] / poly[c][2] + (double)cam.cx;
    pv[c] = (double)cam.fy * poly[c][1] / poly[c][2] + (double)cam.cy;
    umin = fmin(umin, pu[c]); umax = fmax(umax, pu[c]);
    vmin = fmin(vmin, pv[c]); vmax = fmax(vmax, pv[c]);
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

  BinRec b;
  // orientation: make the polygon counter-clockwise (positive signed area)
  double area = 0.0;
  for (int c = 0; c < np; ++c) {
    const int d = (c + 1 == np) ? 0 : c + 1;
    area += pu[c] * pv[d] - pu[d] * pv[c];
  }
  for (int e = 0; e < 5; ++e) b.edge[e][0] = b.edge[e][1] = b.edge[e][2] = 0.0;
  if (np >= 3 && fabs(area) > 1e-3) {
    // signed distance to each edge, positive inside the counter-clockwise polygon
    b.nedge = np;
    for (int e = 0; e < np; ++e) {
      const int ia = area > 0 ? e : np - 1 - e;
      const int ib = area > 0 ? (e + 1 == np ? 0 : e + 1) : (e + 1 == np ? np - 1 : np - 2 - e);
      const double ex = pu[ib] - pu[ia], ey = pv[ib] - pv[ia];
      const double len = sqrt(ex * ex + ey * ey);
      if (!(len > 0.0)) {  // repeated vertex: no constraint
        b.edge[e][0] = 0.0; b.edge[e][1] = 0.0; b.edge[e][2] = 1.0;
        continue;
      }
      b.edge[e][0] = -ey / len;
      b.edge[e][1] = ex / len;
      b.edge[e][2] = (ey * pu[ia] - ex * pv[ia]) / len;
    }
  } else {
    b.nedge = -1;
  }
  // depth lower bound over the grown, clipped rectangle, rounded down.  The
  // ray parameter of a hit equals its camera z only up to the float32
  // rounding of R (R R^T = I to ~1e-7): a relative margin of 4e-6 covers it.
  float tl = __double2float_rd(fmax(zmin, zn) * (1.0 - 4e-6));
  b.tlb = tl;
  b.tx0 = (int)i0 / sl.tile_w; b.tx1 = (int)i1 / sl.tile_w;
  b.ty0 = (int)j0 / sl.tile_h; b.ty1 = (int)j1 / sl.tile_h;
  b.slot = s;
  b.pad[0] = b.pad[1] = b.pad[2] = 0;
  a.brecs[r] = b;
}

}  // namespace

extern "C" int plane_project(const ps_layout* L, void* ws, const float* center, const float* quat,
                             const float* radii, int K, const ps_camera* cams, int n_cams,
                             const float* lambda, const ps_params* prm, void* stream) {
  int rc = ps_check_ws(L, ws, "plane_project");
  if (rc) return rc;
  if (!center || !quat || !radii || !cams || !lambda || !prm)
    return ps_set_error(PS_ERR_INVALID, "plane_project: null pointer");
  if (K < L->n_planes) return ps_set_error(PS_ERR_INVALID, "plane_project: K=%d < planes referenced %d", K, L->n_planes);
  if (n_cams <= 0) return ps_set_error(PS_ERR_INVALID, "plane_project: n_cams <= 0");
  if (!(prm->tau > 0.f && prm->tau < 1.f) || !(prm->z_near > 0.f) || prm->M < 1 || prm->M > kMaxM ||
      (prm->weight_mode != 0 && prm->weight_mode != 1))
    return ps_set_error(PS_ERR_INVALID, "plane_project: bad ps_params");
  if (L->n_records == 0) return PS_OK;
  char* base = (char*)ws;
  ProjArgs a;
  a.slots = (const ps_slot*)(base + L->region[R_SLOTS]);
  a.S = L->n_slots;
  a.R = L->n_records;
  a.center = center; a.quat = quat; a.radii = radii;
  a.cams = cams; a.lambda = lambda; a.n_cams = n_cams;
  a.tau = prm->tau; a.z_near = prm->z_near; a.mode = prm->weight_mode; a.two_sided = prm->two_sided;
  a.recs = (Rec*)(base + L->region[R_REC]);
  a.brecs = (BinRec*)(base + L->region[R_BINREC]);
  hipLaunchKernelGGL(project_kernel, dim3((a.R + 255) / 256), dim3(256), 0, (hipStream_t)stream, a);
  PS_HIP_CHECK(hipGetLastError());
  return PS_OK;
}
