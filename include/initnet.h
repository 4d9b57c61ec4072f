/* Learned plane initializer: C ABI of its HIP kernels (gfx950).
 *
 * Not part of the paper's method (Sec. 3.3 initialises planes from monocular
 * depth); this network proposes planes from back-projected depth samples so
 * that a fit can start closer to the answer.  Per view, N points X [N][3]
 * (camera frame, metres) go through three point-wise layers of width C = 256
 * with ReLU, a max over the points and a linear head to P proposals of 12
 * numbers (center 3, quaternion 4, radii 4, confidence logit 1):
 *   h1 = bf16(relu(X W1 + b1)), h2 = bf16(relu(h1 W2 + b2)),
 *   h3 = bf16(relu(h2 W3 + b3)), g[c] = max_n h3[n][c], out = g Wh + bh.
 * bf16(.) rounds to bfloat16 (nearest even).  Weights are bfloat16 copies of
 * float32 masters; the two 256 x 256 layers and the backward's matrix
 * products run on MFMA (bfloat16 operands, float32 accumulation).
 *
 * Conventions: every pointer is device memory owned by the caller; calls are
 * asynchronous on `stream` (a hipStream_t) and allocate nothing; ws is a
 * caller workspace of the size the matching *_ws function returns (floats,
 * 256-byte aligned).  Return 0 (PS_OK) or PS_ERR_INVALID (null pointer, bad
 * size) / PS_ERR_HIP; the message is ps_last_error().
 */
#ifndef INITNET_H
#define INITNET_H

#include <stddef.h>
#include <stdint.h>

#include "planesplat.h"

#ifdef __cplusplus
extern "C" {
#endif

#define IN_C 256     /* width of the point layers */
#define IN_TM 128    /* points per forward tile: N must be a multiple */
#define IN_OUT 12    /* numbers per proposal */
#define IN_PMAX 256  /* proposals per view, at most */

/* Float32 parameters (masters, gradients, Adam moments), offsets in floats:
 *   W1 [3][C] | b1 [C] | W2 [C][C] | b2 [C] | W3 [C][C] | b3 [C] | Wh [C][12P] | bh [12P]
 * W[i][o] maps input i to output o. */
int64_t initnet_param_count(int P);

/* Bfloat16 copies (uint16 bit patterns), offsets in elements:
 *   W1 [3][C] | W2t [C][C] | W2 [C][C] | W3t [C][C] | Wh [C][12P] | Wht [12P][C]
 * with W2t[o][i] = W2[i][o] (likewise W3t, Wht). */
int64_t initnet_packed_count(int P);

/* Round the masters to the bfloat16 copies (after every optimiser step). */
int initnet_pack(const float* master, int P, uint16_t* packed, void* stream);

/* Forward of B views of N points each.  X [B][N][3]; outputs g [B][C]
 * (pooled features), arg [B][C] (index of the point that attains each
 * maximum, the smallest on ties) and out [B][12P].  dump: NULL, or
 * [3][B*N][C] bfloat16 receiving h1, h2, h3 (testing).  N % IN_TM == 0. */
int initnet_forward(const float* master, const uint16_t* packed, int P, const float* X, int B, int N,
                    float* g, int32_t* arg, float* out, float* ws, uint16_t* dump, void* stream);
int64_t initnet_forward_ws(int B, int N);

/* Set loss of the proposals against target planes and its gradient.
 * tgt [T][11] (center 3, quaternion 4, radii 4; camera frame of the view),
 * the targets of view b being rows tgt_off[b] .. tgt_off[b+1]-1 (tgt_off:
 * device int32 [B+1]).  Per view, with the plane descriptors n (unit normal)
 * and half-extents a >= b:
 *   d(p,t) = |c_p - c_t|^2 + 0.25 (1 - (n_p . n_t)^2) + 0.25 ((a_p-a_t)^2 + (b_p-b_t)^2)
 *   L_b = mean_t min_p d(p,t) + mean_p BCE(conf_p, [p is the nearest proposal of a target])
 * loss [B] receives L_b; d_out [B][12P] the gradient of mean_b L_b. */
int initnet_set_loss(const float* out, int B, int P, const float* tgt, const int32_t* tgt_off, float* loss,
                     float* d_out, void* stream);

/* Gradient of sum_b d_out[b] . out[b] with respect to the float32 parameters
 * (grad, layout of initnet_param_count; overwritten).  X, g, arg as returned
 * by initnet_forward for the same parameters.  The point layers are
 * differentiated only at the B*C points that attain a maximum: their
 * activations are recomputed, no per-point state is kept. */
int initnet_backward(const float* master, const uint16_t* packed, int P, const float* X, int B, int N,
                     const float* g, const int32_t* arg, const float* d_out, float* grad, float* ws,
                     void* stream);
int64_t initnet_backward_ws(int B, int P);

/* Adam with bias correction on n float32 parameters (step: device int32,
 * 1-based). */
int initnet_adam(float* master, float* m, float* v, const float* grad, int64_t n, const int32_t* step,
                 float lr, float beta1, float beta2, float eps, void* stream);

/* Geometry of the per-view form (reading: the network sees N depth samples
 * of one view and proposes P planes in that view's camera frame; the scene
 * initialisation takes from each initial plane's nearest confident proposal
 * its supporting plane).
 *
 * initnet_view_points: the network's input of V views.  depth [V][H][W]
 * (device, metres, 0 = no surface); cams: device array of V ps_camera; cand
 * [V][n_cand] candidate pixel indices (y W + x, drawn by the caller) and eps
 * [V][n_cand] standard normal draws (drawn by the caller).  Per view the
 * candidates are taken in order and the first N with depth > 0 are kept; a
 * kept pixel (i, j) with depth z becomes the camera-frame point z' d_c,
 * z' = z (1 + sigma eps), d_c = ((i + 1/2 - cx) / fx, (j + 1/2 - cy) / fy, 1)
 * (float64, each operation rounded on its own, stored as float32).  With
 * fewer than N valid candidates the kept points repeat in order (zeros if
 * none).  X [V][N][3] (device), n_valid [V] (device): points kept per view. */
int initnet_view_points(const float* depth, const ps_camera* cams, int V, int H, int W, const int32_t* cand,
                        const float* eps, int n_cand, int N, float sigma, float* X, int32_t* n_valid,
                        void* stream);

/* initnet_proposals_to_world: the proposals of B views (out [B][12P], the
 * network's camera-frame output) decoded as the set loss decodes them
 * (center; unit quaternion of (o3 + 1, o4, o5, o6); radii softplus(o) + 0.01;
 * confidence sigmoid(o11)) and mapped to the world frame with the camera of
 * each view (cams[view_cam[b]]): center R^T (c - t), rotation R^T R(q) as a
 * unit quaternion (Shepperd's method).  Outputs [B*P][3], [B*P][4], [B*P][4],
 * [B*P] (device). */
int initnet_proposals_to_world(const float* out, int B, int P, const ps_camera* cams, const int32_t* view_cam,
                               float* center, float* quat, float* radii, float* conf, void* stream);

/* initnet_refine_planes: the learned initialisation of a scene.  For each of
 * the K initial planes (center [K][3], quat [K][4], radii [K][4]) the
 * nearest proposal (Q of them, world frame, from initnet_proposals_to_world)
 * among those with confidence >= conf_min, by the set loss's distance
 * d = |c_p - c_k|^2 + 0.25 (1 - (n_p . n_k)^2) + 0.25 ((a_p - a_k)^2 + (b_p - b_k)^2)
 * (float64, each operation rounded on its own; the smallest index on ties).
 * If d <= d_max the plane takes the proposal's supporting plane: its normal
 * becomes n_p turned to the initial normal's side, its center moves onto
 * that plane along the normal, its frame turns by the smallest rotation that
 * takes the old normal to the new one; radii are kept.  Otherwise the plane
 * is unchanged.  out_center [K][3], out_quat [K][4], match [K] (the
 * proposal index, or -1): device. */
int initnet_refine_planes(const float* center, const float* quat, const float* radii, int K, const float* p_center,
                          const float* p_quat, const float* p_radii, const float* p_conf, int Q, double conf_min,
                          double d_max, float* out_center, float* out_quat, int32_t* match, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* INITNET_H */
