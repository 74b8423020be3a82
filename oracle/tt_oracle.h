/*
 * tt_oracle.h -- FP64 single-threaded CPU oracle for the per-frame deformation solve of
 * H. Zhou and J. Jagadeesan, "Real-time Surface Deformation Recovery from Stereo Videos"
 * (arXiv:2007.08576).
 *
 * TEST INFRASTRUCTURE ONLY. This library exists to check the GPU library against a plain,
 * slow, obviously correct restatement of the paper's method. Only the test suite, the smoke
 * entry point and the benchmark's CPU-baseline leg may load it. It shares no code, header,
 * table or helper with the GPU library, and the GPU library never calls it.
 *
 * Everything is double precision and single threaded. Loops follow the order in which the
 * paper states each step; there is no blocking, fusion or reordering.
 *
 * Units: millimetres and radians. Depth maps are row-major (v * width + u); a depth value that
 * is not finite or not > 0 is invalid. Feature coordinates of NaN mean "no depth".
 *
 * Dual quaternions are 8 doubles [qr.w qr.x qr.y qr.z qd.w qd.x qd.y qd.z]; the node warp maps
 * x -> R(qr) x + t with t = 2 vec(qd * conj(qr)). Increments are node-centred: xi_i = (omega_i,
 * tau_i) in R^6 acts as Delta_i(x) = Exp(omega_i)(x - p_i) + p_i + tau_i with p_i the node's
 * current position, and the new warp is Delta_i composed after W_i.
 *
 * Return codes: 0 success, negative on error (TTO_EINVAL bad argument, TTO_ENOMEM allocation
 * failure, TTO_ESTATE frame before template).
 */
#ifndef TT_ORACLE_H
#define TT_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { TTO_OK = 0, TTO_EINVAL = -1, TTO_ENOMEM = -2, TTO_ESTATE = -3 };

/* How the damped normal equations of an LM step are solved (tto_params.solver).
 * TTO_SOLVE_DENSE: one coupled 6N x 6N system, textbook Cholesky.
 * TTO_SOLVE_NODE: the literal reading of Sec. 2, where each node warp W_i is updated on its own:
 * only the 6 x 6 diagonal block of node i (and its part of J^T r) enters node i's step, each
 * block is factored by Cholesky, and the step is accepted or rejected as a whole. */
enum { TTO_SOLVE_DENSE = 0, TTO_SOLVE_NODE = 1 };

typedef struct {
  int width, height;      /* depth map size in pixels */
  double fx, fy, cx, cy;  /* pinhole: u = fx x / z + cx, v = fy y / z + cy (pixel centres at integers) */
} tto_intrinsics;

typedef struct {
  int num_control_points; /* N, chosen by farthest-point sampling over the template */
  int knn;                /* nodes blended per point (4) */
  double w_orb;           /* weight of the feature term, Eq. (1): 10 */
  double w_angle;         /* Eq. (5): 20 */
  double w_rotation;      /* Eq. (5): 100 */
  double lambda_arap;     /* scale of the dynamic ARAP weight (Sec. 2): 1 */
  double tukey_c;         /* Tukey constant of the ICP term, mm: 5 */
  double H;               /* reweighting threshold of Eq. (4), mm: 3 */
  int ransac_refs;        /* reference matches per frame (Sec. 2.1): 30 */
  int ransac_iters;       /* R / w alternations per reference (Sec. 2.1): 10 */
  int lm_iters;           /* LM iterations per frame: 10 */
  int max_hamming;        /* matches with a larger distance are unusable; 256 keeps all */
  double lm_lambda0;      /* initial Marquardt damping per frame: 1e-4 */
  uint64_t seed;          /* seed of the reference-match sampler */
  int solver;             /* TTO_SOLVE_DENSE or TTO_SOLVE_NODE */
  int arap_knn;           /* 0: ARAP over all pairs of control points (Sec. 2.2, dense); k > 0:
                             only pairs where one node is among the other's k nearest (0..32) */
  int assoc_zbuffer;      /* 0: every deformed template point takes its nearest pixel; 1: of the
                             points that project to one pixel only the nearest to the camera
                             (smallest z as float32, ties to the lower index) takes it */
  int assoc_kdtree;       /* 0: re-projection (Sec. 2); 1: the closest-point alternative the paper
                             contrasts it with -- the nearest target point in 3D (FP64 distance,
                             ties to the lower pixel index) among the pixels with a normal. Not
                             with assoc_zbuffer. */
} tto_params;

typedef struct tto_stream tto_stream;

/* Optional per-frame outputs (each pointer may be NULL). Sizes: K1 template features, M template
 * points, R = ransac_refs, T = lm_iters, n = 6 N. */
typedef struct {
  int32_t* match_idx;     /* [K1] nearest frame feature */
  int32_t* match_dist;    /* [K1] its Hamming distance */
  double* wstar;          /* [K1] pre-selection weight (0 if unusable or never kept) */
  uint8_t* preselected;   /* [K1] 1 if in the pre-selected inlier set */
  int32_t* hyp_k0;        /* [R] reference match of each hypothesis (-1 if not drawn) */
  double* hyp_W;          /* [R] sum of weights after the last reweighting */
  int32_t* hyp_nin;       /* [R] matches with d <= H */
  uint8_t* hyp_kept;      /* [R] 1 if kept, 0 if dropped, 2 if degenerate */
  int32_t* corr0;         /* [M] iteration-0 pixel index of each template point, or -1 */
  double* r0;             /* [M] iteration-0 point-to-plane residual (0 if no correspondence) */
  double* omega0;         /* [M] iteration-0 Tukey weight */
  double* orbw0;          /* [K1] iteration-0 feature weight */
  double* A0;             /* [n*n] iteration-0 J^T J, row-major, undamped */
  double* g0;             /* [n] iteration-0 J^T r */
  double* w_arap;         /* [1] dynamic ARAP weight of this frame */
  double* cost_old;       /* [T] cost at the iterate before the step */
  double* cost_new;       /* [T] cost at the candidate (NaN if the factorisation failed) */
  double* lambda;         /* [T] damping used in the step */
  uint8_t* accepted;      /* [T] 1 if the candidate was accepted */
  double* delta0;         /* [n] iteration-0 step (left unwritten if the factorisation failed) */
  double* w_arap_iter;    /* [T] ARAP weight each iteration's costs and normal equations use */
} tto_frame_debug;

void tto_default_params(tto_params* p);

int tto_create_stream(const tto_params* p, const tto_intrinsics* K, tto_stream** out);
int tto_destroy(tto_stream* s);

/* Template: M points (x,y,z per point), K1 template features with 3D position and 32-byte
 * descriptor. Chooses the control points, blend neighbours and weights, ARAP pair weights;
 * resets all warps to identity and the frame counter to 0. */
int tto_set_template(tto_stream* s, const float* pts_xyz, int M, const float* feat_xyz,
                     const uint8_t* feat_desc, int K1);

/* One frame: depth (H x W), K2 frame features. Writes the deformed template (M x 3) and the node
 * warps (N x 8); either may be NULL. */
int tto_track_frame(tto_stream* s, const float* depth_mm, const float* feat_xyz,
                    const uint8_t* feat_desc, int K2, double* out_vertices, double* out_dq,
                    tto_frame_debug* dbg);

/* Template queries. */
int tto_num_nodes(const tto_stream* s);
int tto_get_template_info(const tto_stream* s, int32_t* node_idx, int32_t* knn_pts,
                          double* alpha_pts, int32_t* knn_feat, double* alpha_feat,
                          double* sbar, double* s_arap);
/* Warp state and frame counter (teacher forcing). */
int tto_get_state(const tto_stream* s, double* dq, int64_t* frame);
int tto_set_state(tto_stream* s, const double* dq, int64_t frame);

/* ---- Step-level entry points used to pin the oracle against the mathematics ---- */

/* Nearest frame descriptor by Hamming distance, ties to the lower index. */
void tto_hamming_match(const uint8_t* desc1, int K1, const uint8_t* desc2, int K2, int32_t* idx,
                       int32_t* dist);

/* argmax_{R in SO(3)} tr(R^T M) for a 3x3 row-major M. Returns 1 if degenerate. */
int tto_rotation_fit(const double* M, double* R, double* sigma);

/* 1-point RANSAC + reweighting pre-selection over K matches o1[k], o2[k] (3 doubles each);
 * usable[k] != 0 marks the matches that take part. refs == 0 means "every usable match is a
 * reference, in index order" (exhaustive); otherwise references are drawn from the sampler with
 * the given seed and frame number. Outputs as in tto_frame_debug; hyp arrays sized
 * max(refs, K). Returns the number of hypotheses. */
int tto_preselect(const double* o1, const double* o2, const uint8_t* usable, int K, double H,
                  int refs, int iters, uint64_t seed, int64_t frame, double* wstar,
                  uint8_t* preselected, int32_t* hyp_k0, double* hyp_W, int32_t* hyp_nin,
                  uint8_t* hyp_kept);

/* Splitmix64 outputs number 1..n of the state seeded with `state`. */
void tto_splitmix64(uint64_t state, int n, uint64_t* out);

/* Target normal map: normals [H*W*3] (0 where invalid) and valid [H*W]. */
void tto_normal_map(const float* depth, const tto_intrinsics* K, double* normals, uint8_t* valid);

/* Dual-quaternion blending of one point p with k nodes (indices into dq), weights alpha. */
void tto_dqb(const double* dq, const int32_t* nodes, const double* alpha, int k, const double* p,
             double* v);

/* Dual-quaternion algebra used by the tests. */
void tto_dq_transform(const double* dq, const double* p, double* out);
void tto_dq_from_rt(const double* qrot, const double* t, double* dq);

/* Apply node-centred increments delta [6N] to warps dq [8N]; result in dq_out. */
int tto_apply_increment(const tto_stream* s, const double* dq, const double* delta, double* dq_out);

/* Frame set-up without solving: normal map, matching and pre-selection for this frame's
 * inputs, kept in the stream for the calls below. Does not advance the frame counter. */
int tto_frame_begin(tto_stream* s, const float* depth_mm, const float* feat_xyz,
                    const uint8_t* feat_desc, int K2);

/* Number of residual rows: M + 3 K1 + 8 N (N - 1). */
int tto_num_rows(const tto_stream* s);

/* Weighted residual vector at warps dq_eval, with correspondences and weights taken at dq_assoc
 * and the ARAP weight w_arap (if w_arap < 0 it is computed from the association at dq_assoc).
 * r [rows]. Optional J [rows * 6N] row-major: analytic Jacobian at dq_eval (same association). */
int tto_residuals(tto_stream* s, const double* dq_eval, const double* dq_assoc, double w_arap,
                  double* r, double* J, double* w_arap_used);

/* Normal equations assembled row by row: A = J^T J [n*n], g = J^T r [n] at dq (association at
 * dq, ARAP weight as in tto_residuals). */
int tto_normal_equations(tto_stream* s, const double* dq, double w_arap, double* A, double* g);

/* Textbook Cholesky A = L L^T (row-major n x n; L written to the lower triangle of L, zeros
 * above). Returns 0, or k+1 if pivot k is not positive. */
int tto_cholesky(const double* A, int n, double* L);
/* Solve L L^T x = b with the factor from tto_cholesky. */
void tto_cholesky_solve(const double* L, int n, const double* b, double* x);

/* ---- Uniform ORB features (Sec. 2.1): FAST corners on the GPU's reading, kept where no
 * neighbouring pixel has a larger corner response, with oriented binary descriptors. ---- */

/* Pixels closer than this to the image border are never keypoints (FAST circle 3, orientation
 * disc 15, rotated pattern + 5x5 box 16). */
#define TTO_ORB_BORDER 18

typedef struct {
  int fast_threshold; /* t: circle pixels brighter than I_p + t or darker than I_p - t (20)   */
  int nms_radius;     /* r: a corner is kept iff its response beats every other corner's in the
                         (2r+1)^2 window around it, ties to the lower pixel index (1)           */
  int max_features;   /* at most this many keypoints, the first in raster order (4096)        */
} tto_orb_params;

void tto_orb_default_params(tto_orb_params* p);

/* FAST-9 corner response of pixel (u, v) of an 8-bit image (row-major, W x H): with the 16
 * pixels of the radius-3 circle, the pixel is a corner iff 9 or more contiguous ones (cyclic)
 * are all brighter than I_p + t or all darker than I_p - t; its response is then
 * max(sum over brighter of (I - I_p - t), sum over darker of (I_p - I - t)), else 0. (u, v)
 * must be at least 3 pixels from the border. */
int tto_fast_response(const uint8_t* img, int W, int u, int v, int t);

/* Keypoints, 3D points and descriptors of an 8-bit image.
 *   kp [max][2] (u, v), raster order; xyz [max][3]: the back-projected depth at the keypoint
 *   (NaN if depth is NULL or the pixel's depth is invalid); desc [max][32]: bit k (byte k/8,
 *   bit k%8 from the least significant) = 1 iff S(p + a_k) < S(p + b_k), with S the 5x5 box
 *   sum of the image and (a_k, b_k) = pattern row k = (x1, y1, x2, y2) rotated to the
 *   keypoint's orientation bin; angle_bin [max] in 0..29: the intensity-centroid angle
 *   atan2(m01, m10) over the disc of radius 15, in 12-degree bins rounded to nearest.
 *   count[0] = keypoints written, count[1] = corners kept before the max_features cap.
 * K may be NULL when depth is NULL. Returns 0 or TTO_EINVAL / TTO_ENOMEM. */
int tto_orb_detect(const uint8_t* img, int W, int H, const float* depth, const tto_intrinsics* K,
                   const int8_t* pattern, const tto_orb_params* p, int32_t* kp, float* xyz,
                   uint8_t* desc, int32_t* angle_bin, int32_t* count);

#ifdef __cplusplus
}
#endif

#endif
