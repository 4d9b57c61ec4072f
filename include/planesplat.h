/*
 * planesplat.h -- C ABI of the MI355X (gfx950) splatting library for
 * rectangular plane primitives (PlanarSplatting, arXiv 2412.03451).
 *
 * What the library computes.  A plane primitive is a rectangle with center
 * p in R^3, rotation quaternion q = (w, x, y, z) and four radii
 * (r^{x+}, r^{x-}, r^{y+}, r^{y-}) (Sec. 3.1, Eq. 1-3).  For every pixel ray of
 * a pinhole camera, every plane is intersected (Eq. 4), the intersection gets
 * the rectangle splat weight w (Eq. 6-9, steepness lambda of Eq. 10), hits
 * with w >= tau are ordered near to far, the first M are composited front to
 * back into a depth and a normal map (Eq. 11-13), the maps are compared with
 * targets by the loss of Eq. 14, gradients flow back to (p, q, r) and an Adam
 * step updates them (Sec. 3.3).
 *
 * Readings where the paper is silent or garbled (shared with the tests):
 *   - Eq. 4 is read as t = ((p - o) . n) / (d . n);
 *   - the ray of pixel (i, j) passes through (i + 1/2, j + 1/2); its camera
 *     frame direction has z = 1, so t is the camera z-depth;
 *   - weight_mode 0: w = min(1, 2 sigmoid(5 lambda a*)) (the printed 2 sigma,
 *     clamped: the rectangle interior is opaque); weight_mode 1:
 *     w = sigmoid(5 lambda a*); a* = min(a_X, a_Y), a_X = r^{x+/-} - |P_X|;
 *   - a hit needs |d . n| > 1e-12 |d| and t > z_near;
 *   - per-ray order: depth rounded to float32, ties by plane index;
 *   - the rendered normal is the camera-frame plane normal flipped to face
 *     the camera (two_sided = 1) or R(q) e_z as is (two_sided = 0);
 *   - a pixel without hits renders depth 0 and normal 0.
 *
 * Conventions for every call.
 *   - Pointers documented "device" are device memory the caller owns; the
 *     library never allocates or frees.  Scratch lives in one caller-owned
 *     workspace of ps_layout.ws_bytes bytes (256-byte aligned).
 *   - `stream` is a hipStream_t passed as void*.  Calls are asynchronous on it
 *     and capturable in a HIP graph, except where a call says it synchronises.
 *   - Return value: PS_OK, or an error code with a message from
 *     ps_last_error() (thread-local).  Invalid arguments are rejected before
 *     any launch.
 *   - Float arrays are float32.  Plane parameters are row-major [K][3]
 *     (center), [K][4] (quat, w first), [K][4] (radii: x+, x-, y+, y-).
 *   - A "job" (ps_slot) renders the planes [plane_begin, plane_end) with one
 *     camera into one image.  Several jobs form a batch (several views of one
 *     scene, or several scenes).  Depth of job s occupies
 *     depth[pix_off, pix_off + H*W) row-major; its normal occupies
 *     normal[3*pix_off, 3*pix_off + 3*H*W) as three [H][W] planes (x, y, z).
 */
#ifndef PLANESPLAT_H
#define PLANESPLAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PS_OK 0
#define PS_ERR_INVALID 1   /* bad argument (null pointer, bad size, bad tile shape) */
#define PS_ERR_CAPACITY 2  /* more (tile, plane) pairs than the workspace holds   */
#define PS_ERR_HIP 3       /* a HIP runtime call failed                            */

/* Pinhole camera; x_cam = R x_world + t, OpenCV axes (x right, y down,
 * z forward), pixel (i, j) center at (i + 1/2, j + 1/2).  80 bytes. */
typedef struct ps_camera {
  int32_t width, height;
  float fx, fy, cx, cy;
  float R[9]; /* row-major world->camera rotation */
  float t[3];
  int32_t pad[2];
} ps_camera;

/* Method constants (Sec. 3.2).  Paper values: M = 30, tau = 1e-4. */
typedef struct ps_params {
  int32_t M;           /* nearest hits composited per ray, 1..30 */
  float tau;           /* weight filter, 0 < tau < 1 */
  float z_near;        /* near clip in metres, > 0 */
  int32_t weight_mode; /* 0: min(1, 2 sigmoid), 1: sigmoid, 2: the Gaussian of Eq. 5
                          (planar, standard deviations the radii of the hit's side) */
  int32_t two_sided;   /* 1: normals face the camera */
  int32_t flags;       /* bit 0: force the exact fallback ordering path (testing);
                          bits 4-5: pending hits kept per lane by the render
                          walks, 0: 6, 1: 4, 2: 8, 3: 12 (a tuning knob, the
                          result does not depend on it);
                          bit 6: record per-block walk statistics of the
                          forward and backward renders (ps_read_counters
                          out[6..17] and out[19]);
                          bit 7: plane_render_fwd adds 256 to the hit count
                          (its `count` output) of every pixel that took the
                          exact fallback ordering path;
                          bit 9: the forward's launch may be persistent too
                          (by default only the backward's is: measured);
                          bit 8: the render calls launch one workgroup per 8x8
                          block even when the blocks are more than four times
                          what the GPU holds resident (by default such a
                          backward launch is persistent:
                          resident workgroups claim blocks from an atomic work
                          queue, longest lists first; same results);
                          bit 10: the backward's per-plane reduction takes a
                          wave per plane at any plane count (by default from
                          8192 planes on, below that a workgroup per plane;
                          the same summation order, so the same bits) */
} ps_params;

/* One render job.  The caller fills the first block; ps_layout_init fills
 * the second.  64 bytes. */
typedef struct ps_slot {
  int32_t plane_begin, plane_end; /* planes [begin, end) of the plane arrays */
  int32_t cam;                    /* camera index of the job */
  int32_t width, height;          /* image size of the job's camera */
  int32_t tile_w, tile_h;         /* binning tile: 8x8, 16x16 or 32x8 */
  int32_t scene;                  /* scene index (loss is reported per job) */
  int32_t tiles_x, tiles_y;       /* filled: tiles per row / column */
  int32_t rec_begin;              /* filled: first projection record */
  int32_t tile_begin;             /* filled: first tile */
  int32_t item_begin;             /* filled: first 8x8 render item */
  int32_t pad;
  int64_t pix_off;                /* filled: first pixel of the job */
} ps_slot;

/* Sizes and workspace carving of a batch of jobs (host struct). */
#define PS_NUM_REGIONS 24
typedef struct ps_layout {
  int32_t n_slots;
  int32_t n_records;   /* sum of (plane_end - plane_begin) */
  int32_t n_tiles;
  int32_t n_items;     /* 8x8 pixel blocks */
  int64_t n_pixels;
  int64_t pair_capacity;
  int32_t max_sub;     /* 8x8 blocks per tile, maximum over jobs */
  int32_t n_planes;    /* planes referenced: max plane_end */
  int32_t max_items;   /* 8x8 blocks of the largest job */
  int32_t max_chunks;  /* groups of 64 tiles of the largest job */
  int32_t slots_sorted; /* plane_begin and plane_end nondecreasing over the slots */
  int32_t pad;
  size_t region[PS_NUM_REGIONS]; /* byte offsets inside the workspace */
  size_t ws_bytes;
} ps_layout;

/* Fill the derived fields of slots[0..n_slots) (host array, modified in
 * place) and compute the layout for at most pair_capacity (tile, plane)
 * pairs.  Tile shapes must be 8x8, 16x16 or 32x8; sizes must be positive. */
int ps_layout_init(ps_slot* slots, int n_slots, int64_t pair_capacity, ps_layout* out);

/* Workspace bytes for a layout (same as out->ws_bytes). */
size_t ps_workspace_bytes(const ps_layout* L);

/* Copy the slot table into the device workspace `ws` (ps_layout.ws_bytes
 * bytes, device, 256-byte aligned) and clear its counters.  Call once per
 * workspace, and again after changing the host slots. */
int ps_workspace_init(const ps_layout* L, const ps_slot* slots, void* ws, void* stream);

/* Device-side change of the camera of every job: cam[s] = view_of_slot[s]
 * (device int array of n_slots), for captured fitting steps. */
int ps_set_cameras(const ps_layout* L, void* ws, const int32_t* view_of_slot, void* stream);

/* plane_render_fwd_loss: plane_render_fwd and loss_depth_normal_cam
 * (Eq. 11-14) in one pass: the forward forms the loss of every pixel it
 * renders right after compositing it, with the arithmetic of the loss call,
 * so depth, normal, g_depth, g_normal and loss hold the same bits as the two
 * calls give (the loss kernel's read of the maps is saved).  Arguments as in
 * the two calls; tgt_off may be null (targets laid out like the jobs, as for
 * loss_depth_normal), else n_tgt offsets as n_cams of loss_depth_normal_cam.
 * loss may be NULL: the per-block partial sums then stay in the workspace
 * and plane_render_bwd_adam forms the sums. */
int plane_render_fwd_loss(const ps_layout* L, void* ws, const ps_camera* cams, int n_cams, const float* lambda,
                          const ps_params* prm, float* depth, float* normal, const float* tgt_depth,
                          const float* tgt_normal, const uint8_t* mask, const int64_t* tgt_off, int n_tgt,
                          float a_cos, float a_nl1, float a_d, float* loss, float* g_depth, float* g_normal,
                          void* stream);

/* The list-storing variant of the render pair, kept to compare memory with
 * the recompute backward above (it is not used by the fitting loop).
 * plane_render_fwd_lists renders like plane_render_fwd and also stores, for
 * every pixel p and committed hit j < M, list_pos[j * n_pixels + p] (the
 * hit's position in its tile list), list_a[...] (its a*) and list_T[...]
 * (transmittance in front of it), and list_count[p] (device buffers of
 * M * n_pixels int32 / float / float and n_pixels int32; entries j >=
 * list_count[p] are left untouched).  plane_render_bwd_lists computes the
 * gradients of plane_render_bwd from those lists instead of recomputing each
 * pixel's sequence; it needs the workspace of the same tile_bin. */
int plane_render_fwd_lists(const ps_layout* L, void* ws, const ps_camera* cams, int n_cams,
                           const float* lambda, const ps_params* prm, float* depth, float* normal,
                           int32_t* list_pos, float* list_a, float* list_T, int32_t* list_count, void* stream);
int plane_render_bwd_lists(const ps_layout* L, void* ws, const float* center, const float* quat,
                           const float* radii, int K, const ps_camera* cams, int n_cams, const float* lambda,
                           const ps_params* prm, const float* g_depth, const float* g_normal,
                           const int32_t* list_pos, const float* list_a, const int32_t* list_count,
                           float* g_center, float* g_quat, float* g_radii, void* stream);

/* Plane splitting (Sec. 3.3).  plane_grad_accumulate adds |g_radii| to acc
 * (device float [K][4]) and 1 to cnt[k] (device int32 [K]) for every plane
 * whose radii gradient is not all zero (the plane took part in the
 * iteration's render); the caller clears both after each split.
 * plane_split averages the radii gradients over the iterations each plane
 * took part in, as the gradient of the per-pixel mean loss: with
 * gx = (acc[k][x+] + acc[k][x-]) * scale[k] and ct = 2 cnt[k] (float32),
 * plane k is cut across its X extent (two halves side by side along its X
 * axis, each with both X radii a quarter of the extent) when
 * gx > thresh * ct, likewise across Y; both gives four children (a plane
 * with cnt[k] <= 0 is kept).  scale:
 * device float [K], the factor from the accumulated loss to the per-pixel
 * mean (1 / pixels per view of the plane's scene for the summed loss of
 * loss_depth_normal), or NULL for 1.  The rotation is kept and so are the
 * radii along an axis that is not cut.  Children of plane k are consecutive
 * and in plane order (x- half before x+, then y- before y+) at
 * out_* [first[k], first[k+1]) with parent[] = k; first: device int32
 * [K + 1], first[K] = *k_out (device int32) = the new plane count.  out_*:
 * device float [4K][3], [4K][4], [4K][4]; parent: int32 [4K]; ws: device
 * int32 [K + 1]. */
int plane_grad_accumulate(const float* g_radii, float* acc, int32_t* cnt, int K, void* stream);
int plane_split(const float* center, const float* quat, const float* radii, const float* acc, const int32_t* cnt,
                const float* scale, float thresh, int K, float* out_center, float* out_quat, float* out_radii,
                int32_t* parent, int32_t* first, int32_t* k_out, int32_t* ws, void* stream);

/* Scene initialisation from depth (Sec. 3.1): plane centers are random
 * points of a coarse surface built from the depth maps, radii half the
 * distance to the nearest other center, rotation from the surface normal.
 *
 * depth_points fuses the maps into one point per occupied voxel.  Inputs:
 * depth [V][H][W] and normal [V][3][H][W] (device float32, camera-frame
 * normals, the layouts plane_render_fwd writes), cams: device array of V
 * ps_camera (intrinsics and pose; their width and height are not read, the
 * maps are H x W).  Every stride-th pixel (rows and columns from 0) counts
 * when depth > 0 and |N| >= 0.5; its point is R^T (z d_c - t) with
 * z = depth / |N|, d_c = ((i + 1/2 - cx) / fx, (j + 1/2 - cy) / fy, 1), its
 * normal R^T N / |N|; float64 arithmetic, each operation rounded (no fused
 * multiply-add).  Voxel index floor(x / voxel) per axis (grid anchored at the
 * origin; a pixel whose index has magnitude >= 2^20 on an axis is dropped).
 * Each occupied voxel keeps the point and normal of its first pixel in
 * (view, row, column) order and voxels are numbered in that order.  Outputs:
 * points and normals [cap][3] (device float32): the first min(n, cap)
 * voxels; *n_out (device int32) = n, the number of occupied voxels.  ws:
 * device scratch of depth_points_ws_bytes(V, H, W, stride) bytes.
 * PS_ERR_INVALID: null pointer, V, H, W or stride < 1, voxel <= 0, cap < 0,
 * ws_bytes too small, or more than 2^29 sampled pixels. */
size_t depth_points_ws_bytes(int V, int H, int W, int stride);
int depth_points(const float* depth, const float* normal, const ps_camera* cams, int V, int H, int W, int stride,
                 float voxel, float* points, float* normals, int cap, int32_t* n_out, void* ws, size_t ws_bytes,
                 void* stream);

/* plane_init_points: K >= 2 planes on the points sel[k] (device int32 [K],
 * indices into points/normals [n][3], device float32; the caller draws
 * them).  center = points[sel[k]]; all four radii max(0.5 d, r_min) with d
 * the distance to the nearest other selected point; quat (w, x, y, z) the
 * shortest rotation taking e_z to normals[sel[k]] (a normal opposite to e_z
 * gives the half turn about X); float64 arithmetic as in depth_points.  An
 * index outside [0, n) gives that plane NaN parameters and is not read.
 * Outputs center [K][3], quat [K][4], radii [K][4] (device float32).
 * PS_ERR_INVALID: null pointer, K < 2, n < 1. */
int plane_init_points(const float* points, const float* normals, int n, const int32_t* sel, int K, float r_min,
                      float* center, float* quat, float* radii, void* stream);

/* plane_init_sphere: the sphere initialisation of the ablation (Sec. 4.3).
 * Bounding sphere of points [n][3] (device float32, n >= 1): center c = the
 * middle of their axis-aligned box, radius R = the largest distance from c
 * to a point.  Plane k sits at c + R u_k, u_k = dirs[k] / |dirs[k]| (device
 * float32 [K][3], drawn by the caller), its normal -u_k (rotation as in
 * plane_init_points), all radii `radius` (0.05 in the paper).  ws: device
 * scratch of 64 bytes.  PS_ERR_INVALID: null pointer, n < 1, K < 1. */
int plane_init_sphere(const float* points, int n, const float* dirs, int K, float radius, float* center,
                      float* quat, float* radii, void* ws, void* stream);

/* plane_merge (Sec. 3.3, plane merge): plane instances of K fitted planes.
 * Planes i and j are related when |d| > cos_thr and |o_i - sign(d) o_j| <
 * off_thr, with d = n_i . n_j, n = R(q / |q|) e_z (Eq. 3; primitives are
 * two-sided, hence the sign) and o = (p - c) . n the offset of the plane
 * from the scene center c (float64, each operation rounded on its own, in
 * this order).  Instances are the connected components of the relation;
 * label[k] is the smallest plane index of plane k's instance and *n_out the
 * number of instances.  The paper's thresholds: cos_thr = cos(25 deg),
 * off_thr = 0.001 m.  center [K][3], quat [K][4], scene_center [3]: device
 * float32; label: device int32 [K]; n_out: device int32; ws: device scratch
 * of plane_merge_ws_bytes(K) bytes.  Runs rounds of linking until a round
 * links nothing (at most K; the stream is synchronised after each round, so
 * the call is not capturable in a graph).  PS_ERR_INVALID: null pointer,
 * K < 1, off_thr < 0, ws_bytes too small. */
size_t plane_merge_ws_bytes(int K);
int plane_merge(const float* center, const float* quat, int K, const float* scene_center, double cos_thr,
                double off_thr, int32_t* label, int32_t* n_out, void* ws, size_t ws_bytes, void* stream);

/* Device-side bookkeeping of one iteration of the fitting loop (Sec. 3.3,
 * Eq. 10), so that whole steps can be captured in a graph and replayed with
 * no host work.  Reads the iteration counter *ite (device int32, 0-based),
 * writes lambda[0] = min(20 exp(-(1 - 0.001 ite)), 300) (Eq. 10, device
 * float), step[0] = ite + 1 (device int32, the 1-based Adam step) and the
 * camera of every job, cam[s] = table[(ite mod n_rows) * n_slots + s]
 * (device int32 [n_rows][n_slots], the view schedule), then increments *ite.
 * Call before plane_project. */
int ps_fit_schedule(const ps_layout* L, void* ws, int32_t* ite, const int32_t* table, int n_rows,
                    float* lambda, int32_t* step, void* stream);

/* plane_project (Sec. 3.1 Eq. 2-3, Sec. 3.2 Eq. 4 and 6): per (plane, job)
 * record in the job's camera frame: normalised rotation, plane offset, the
 * three affine-in-pixel numerators/denominator of t, P_X, P_Y (float64), the
 * camera-facing normal, and the screen footprint of the rectangle grown by
 * the fringe margin delta(lambda) outside which w < tau.
 *   center [K][3], quat [K][4], radii [K][4]: device, K >= layout.n_planes
 *   (K = 0, every job empty: the arrays may be null and nothing is projected);
 *   cams: device array of n_cams ps_camera; lambda: device float scalar;
 *   prm: host struct.  Result lives in the workspace.  The same launch
 *   clears the per-record and per-tile counts that tile_bin accumulates, so
 *   every tile_bin follows a plane_project on the same workspace. */
int plane_project(const ps_layout* L, void* ws, const float* center, const float* quat,
                  const float* radii, int K, const ps_camera* cams, int n_cams,
                  const float* lambda, const ps_params* prm, void* stream);

/* tile_bin (serves the per-ray depth order of Sec. 3.2: each ray's surviving
 * intersections are sorted by depth, and the sorted per-tile lists let the
 * render commit every hit in exact per-ray order; the footprint tested per
 * tile is the region where the weight of Eq. 7-9 reaches tau): (tile, plane)
 * pairs of every job, each pair keyed by a depth
 * lower bound of the plane over the tile, sorted per tile by (bound, record).
 * Steps: per-record tile count -> wave64 prefix scan of tile and record
 * counts -> key emission -> per-tile sort (LDS bitonic).  If pairs_needed is
 * non-null the call synchronises the stream, stores the number of pairs and
 * returns PS_ERR_CAPACITY when it exceeds layout.pair_capacity (the binning
 * is then incomplete and the render calls write nothing).  A tile may hold at
 * most 32767 pairs (lists longer than 4096 sort in 4096-pair chunks that are
 * then merged).  Without pairs_needed the overflow is only flagged on the
 * device (ps_read_counters).  Call after plane_project (which clears the
 * counts this call accumulates). */
int tile_bin(const ps_layout* L, void* ws, int64_t* pairs_needed, void* stream);

/* plane_render_fwd (Eq. 4, 6-9, 11-13): depth [n_pixels] and normal
 * [3*n_pixels] (device, overwritten, layout above).  trans [n_pixels] (final
 * transmittance) and count [n_pixels] (hits composited) are optional
 * diagnostics (device or NULL).  The per-ray order is exact: hits are
 * committed only once no later candidate of the tile list can be nearer, with
 * an exact per-pixel selection fallback.  cams as for plane_project; the
 * jobs' camera indices must be < n_cams. */
int plane_render_fwd(const ps_layout* L, void* ws, const ps_camera* cams, int n_cams,
                     const float* lambda, const ps_params* prm, float* depth, float* normal,
                     float* trans, int32_t* count, void* stream);

/* plane_render_fwd_noalloc: for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  plane_project -> tile_bin -> plane_render_fwd of ONE job (all
 * K planes, one camera, one width x height image, one tile shape) with the
 * workspace in a static device array of the library instead of a caller
 * buffer; the call allocates nothing and synchronises nothing.
 *   center [K][3], quat [K][4], radii [K][4], cam (one ps_camera), lambda
 *   (scalar): device; prm: host; depth [H*W], normal [3*H*W]: device,
 *   overwritten with the bits plane_render_fwd gives for the same job;
 *   status: device int32 or NULL, set to PS_OK, or to PS_ERR_CAPACITY when
 *   the (tile, plane) pairs exceed what the array holds (depth and normal
 *   are then zero).
 * Limits: the array holds PS_NOALLOC_SCRATCH_BYTES (64 MiB) per GPU, from the
 * library's load until the process ends; the pair capacity is what remains
 * after the per-plane and per-tile regions (about 160 000 pairs for 16x16
 * tiles at 640x480 and K = 2000, twice that for 8x8 tiles).  Sizes whose
 * fixed regions alone exceed the array are rejected with PS_ERR_INVALID
 * before any launch.  Every call on one GPU uses that GPU's one array and
 * leaves its contents behind; each call clears what it needs itself, so calls
 * in sequence are independent, but calls that overlap on one GPU (other
 * streams, other threads) race on the array and must be serialised by the
 * caller.  The stream's device decides which copy of the array is used. */
#define PS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int plane_render_fwd_noalloc(const float* center, const float* quat, const float* radii, int K,
                             const ps_camera* cam, int width, int height, int tile_w, int tile_h,
                             const float* lambda, const ps_params* prm, float* depth, float* normal,
                             int32_t* status, void* stream);

/* loss_depth_normal (Eq. 14): per pixel a_cos |1 - N.N^| + a_nl1 ||N - N^||_1
 * + a_d |D - D^| with its gradient g_depth [n_pixels], g_normal [3*n_pixels]
 * (device, overwritten; sgn(0) = 0).  mask: device uint8 [n_pixels] or NULL.
 * loss: device float [n_slots][4] = the three weighted sums and the plain sum
 * of |D - D^| per job (deterministic). */
int loss_depth_normal(const ps_layout* L, void* ws, const float* depth, const float* normal,
                      const float* tgt_depth, const float* tgt_normal, const uint8_t* mask,
                      float a_cos, float a_nl1, float a_d, float* loss, float* g_depth,
                      float* g_normal, void* stream);

/* loss_depth_normal_cam: as loss_depth_normal, with the targets of every
 * camera in one array, for fitting loops whose view schedule lives on the
 * device (ps_fit_schedule): job s with camera c reads tgt_depth[tgt_off[c] +
 * p] and tgt_normal[3 tgt_off[c] + k H W + p] (p = y W + x, channel k) and
 * mask[tgt_off[c] + p]; the target of camera c has the size of the jobs that
 * use it.  tgt_off: device int64 [n_cams].  A job whose camera index is out
 * of range gets zero loss and gradient. */
int loss_depth_normal_cam(const ps_layout* L, void* ws, const float* depth, const float* normal,
                          const float* tgt_depth, const float* tgt_normal, const uint8_t* mask,
                          const int64_t* tgt_off, int n_cams, float a_cos, float a_nl1, float a_d,
                          float* loss, float* g_depth, float* g_normal, void* stream);

/* plane_render_bwd (the adjoint of Eq. 4-13: ray-plane intersection, splat
 * weight and front-to-back compositing, chained to the primitive's
 * parameters through Eq. 1-3): gradient of sum_px g_depth*D + g_normal.N with
 * respect to center, quat, radii (device [K][3], [K][4], [K][4], overwritten; summed
 * over the jobs that use a plane).  Recomputes each pixel's ordered hit list
 * (no per-pixel list is stored between calls), walks it back to front for the
 * compositing adjoint, reduces per (tile, plane) and chains to (p, q, r) in a
 * fixed order (bitwise deterministic).  Inputs as for plane_project (with
 * K = 0 the plane and gradient arrays may be null). */
int plane_render_bwd(const ps_layout* L, void* ws, const float* center, const float* quat,
                     const float* radii, int K, const ps_camera* cams, int n_cams,
                     const float* lambda, const ps_params* prm, const float* g_depth,
                     const float* g_normal, float* g_center, float* g_quat, float* g_radii,
                     void* stream);

/* plane_render_bwd_adam: plane_render_bwd followed by adam_step_planes
 * (the adjoint of Eq. 4-13, then Sec. 3.3's optimiser step) in one call,
 * with the loss sums of Eq. 14 formed by workgroups added to the backward's
 * per-plane reduction.  Arguments as in the two calls (center,
 * quat, radii are updated in place; g_center, g_quat, g_radii receive the
 * gradients; m, v, step as for adam_step_planes); the results are the bits
 * of the two calls.  loss: device float [n_slots][4] or NULL; if given, the
 * loss sums of the last plane_render_fwd_loss called with a NULL loss (its
 * per-block partials wait in the workspace) are formed here, with the bits
 * that call would have given, and the forward's own reduction launch is
 * saved.  With fewer than 8192 planes (a workgroup per plane in the
 * reduction, ps_params.flags bit 10 clear) the reduction applies the update
 * itself, one launch fewer; with more the update is a kernel of its own:
 * inside a wave-per-plane reduction its latency (two float64 powers, the
 * parameter reads) would lengthen every round of waves.  plane_render_step does the
 * work of plane_render_fwd_loss and this call with one render launch; this
 * call is the step's form with a separate forward. */
int plane_render_bwd_adam(const ps_layout* L, void* ws, float* center, float* quat, float* radii, int K,
                          const ps_camera* cams, int n_cams, const float* lambda, const ps_params* prm,
                          const float* g_depth, const float* g_normal, float* g_center, float* g_quat,
                          float* g_radii, float* m, float* v, const int32_t* step, float lr_center, float lr_quat,
                          float lr_radii, float beta1, float beta2, float eps, float r_min, float* loss,
                          void* stream);

/* plane_render_step: one fitting step's render work in one call, for the
 * loss of Eq. 14: plane_render_fwd_loss (Eq. 11-14) and plane_render_bwd_adam
 * (the adjoint of Eq. 4-13, Sec. 3.3's update, the loss sums), with the
 * forward, the loss and the backward of each 8x8 block in the same launch.
 * The block's walk over its tile list is done once: it composites depth and
 * normal and records, in the block's LDS, the list position of every
 * committed hit; the pixel's loss gradient is formed right after
 * compositing and stays in registers; the backward then commits the hits
 * again from those positions (no per-pixel list leaves the block) and forms
 * the gradients.  depth, normal, g_depth, g_normal, loss, the gradients and
 * the updated planes and Adam moments hold the bits of the two calls.
 * Arguments as in plane_render_fwd_loss (depth, normal, targets, mask,
 * tgt_off, n_tgt, loss weights, g_depth and g_normal as outputs) and
 * plane_render_bwd_adam (planes updated in place, gradients, Adam state and
 * rates; loss: device float [n_slots][4] or NULL).  depth and normal may
 * both be NULL, and g_depth and g_normal both NULL: those outputs are then
 * not written (a fitting loop needs none of them).  ps_params.flags bit 6
 * (walk statistics) is refused: the separate calls record them. */
int plane_render_step(const ps_layout* L, void* ws, float* center, float* quat, float* radii, int K,
                      const ps_camera* cams, int n_cams, const float* lambda, const ps_params* prm, float* depth,
                      float* normal, const float* tgt_depth, const float* tgt_normal, const uint8_t* mask,
                      const int64_t* tgt_off, int n_tgt, float a_cos, float a_nl1, float a_d, float* g_depth,
                      float* g_normal, float* g_center, float* g_quat, float* g_radii, float* m, float* v,
                      const int32_t* step, float lr_center, float lr_quat, float lr_radii, float beta1, float beta2,
                      float eps, float r_min, float* loss, void* stream);

/* adam_step_planes (Sec. 3.3): bias-corrected Adam on the K planes.
 * m, v: device [11*K] laid out as center (3K) | quat (4K) | radii (4K).
 * step: device int, the 1-based step number read by the kernel.  After the
 * update radii are clamped to >= r_min.  Quaternions are not renormalised.
 * K = 0 does nothing (the arrays may then be null). */
int adam_step_planes(float* center, float* quat, float* radii, const float* g_center,
                     const float* g_quat, const float* g_radii, float* m, float* v, int K,
                     const int32_t* step, float lr_center, float lr_quat, float lr_radii,
                     float beta1, float beta2, float eps, float r_min, void* stream);

/* plane_tie_radii: the single-direction radii variant of the ablation
 * (Sec. 4.3, plane radii): each axis has one radius shared by both
 * directions, r^{x+} = r^{x-} and r^{y+} = r^{y-}.  The gradient of a shared
 * radius is the sum of the two directions' gradients; it is written to both
 * entries of g_radii (device float [K][4], 16-byte aligned) so that Adam,
 * started from equal radii, keeps them equal.  Call between
 * plane_render_bwd and adam_step_planes. */
int plane_tie_radii(float* g_radii, int K, void* stream);

/* Counters of the last binning and renders (synchronises the stream):
 * out[0] pairs needed, out[1] overflow flag, out[2] largest tile list,
 * out[3] pixels that took the exact fallback ordering path, out[4] tiles
 * sorted by the large-list pass, out[5] extra backward recompute passes.
 * Statistics of the last forward run with flags bit 6 (per 8x8 block,
 * reduced in a fixed order): out[6] (pixel, candidate) pairs evaluated,
 * out[7] hits composited, out[8] candidate steps summed over blocks, out[9]
 * the most steps of one block, out[10] block run time summed and out[11] its
 * maximum, in ticks of the 100 MHz device wall clock.  Of the last backward
 * run with flags bit 6: out[12..15] the blocks' time spent in set-up,
 * recompute walks, the back-to-front pass with its sort and the gradient pass
 * (ticks, summed), out[16] the candidates visited and out[17] the candidate
 * groups fetched by the gradient pass.  out[18] is nonzero once any tile_bin since
 * ps_workspace_init overflowed (steps replayed from a graph check it after a
 * run of steps); out[19] is the longest backward block time (ticks, flags
 * bit 6).  PS_N_COUNTERS values are written. */
#define PS_N_COUNTERS 20
int ps_read_counters(const ps_layout* L, void* ws, int64_t out[PS_N_COUNTERS], void* stream);

/* Opt-in check for NaN and infinity (the other calls never test their
 * inputs).  Counts the non-finite values among x[0..n) (device, float32) into
 * *d_count (device, caller-owned int64; the call clears it first, with a
 * kernel, so the call may be captured in a graph).  With h_count non-null the
 * count is also copied to *h_count and the stream is synchronised.
 * PS_ERR_INVALID for n < 0, a null d_count, or a null x with n > 0. */
int ps_check_finite(const float* x, int64_t n, int64_t* d_count, int64_t* h_count, void* stream);

/* Issue-rate probe of the vector ALU (measurement only, not a step of the
 * method).  The render kernels' roofline counts lane operations against the
 * non-packed issue rate; this launch measures that rate.  kind 0: fp32,
 * kind 1: fp64.  `blocks` workgroups of 256 lanes each run `iters` rounds of
 * 8 independent fused multiply-adds, so one launch performs
 * blocks * 256 * iters * 8 lane operations; time it with events on `stream`.
 * Every lane writes one value of the chain sum to `sink` (device,
 * blocks * 256 elements of 4 or 8 bytes, caller-owned; sink_bytes is checked).
 * PS_ERR_INVALID for a bad kind, size or pointer. */
int ps_valu_probe(int kind, int blocks, int iters, void* sink, size_t sink_bytes, void* stream);

/* Message of the last error on this thread. */
const char* ps_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PLANESPLAT_H */
