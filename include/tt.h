/*
 * tt.h -- C ABI of the MI355X (gfx950) per-frame deformation solve of
 * H. Zhou and J. Jagadeesan, "Real-time Surface Deformation Recovery from Stereo Videos"
 * (arXiv:2007.08576).
 *
 * The problem (Sec. 2): a template surface, made from the first stereo frame, carries N sparse
 * control points, each with a dual-quaternion warp W_i; the template follows the blend of its
 * neighbouring control points. For every new frame (a depth map from stereo matching plus ORB
 * features with 3D positions) the library estimates all W_i by Levenberg-Marquardt on
 *   f_ICP + w_ORB f_ORB + w_ARAP f_ARAP                                    (Eq. 1)
 * with projective point-to-plane ICP under Tukey's penalty (Sec. 2), ORB matches weighted by
 * the 1-point RANSAC + reweighting pre-selection (Sec. 2.1, Eqs. 2-4) and the dense-connection
 * as-rigid-as-possible cost (Sec. 2.2, Eqs. 5-6).
 *
 * Conventions. Millimetres and radians. Depth maps are row-major float32 (index v*width + u);
 * a value that is not finite or not > 0 is invalid. Pixel centres sit at integer (u, v), and a
 * camera-frame point projects to u = fx x / z + cx, v = fy y / z + cy. 3D points are packed
 * x, y, z float32 triples. ORB descriptors are 32 bytes (256 bits) each. Dual quaternions are
 * [qr.w qr.x qr.y qr.z qd.w qd.x qd.y qd.z], mapping x -> R(qr) x + 2 vec(qd conj(qr)), with
 * qr.w >= 0.
 *
 * Ownership. Host-pointer arguments are caller-owned and used only during the call; the
 * library keeps no caller pointer. A stream and everything resident on the device for it
 * (template, blend tables, descriptors, warps, scratch) are owned by the library until
 * tt_destroy. Device-pointer arguments (tt_track_frame_device) must stay valid until the work
 * queued on the stream's HIP stream has completed.
 *
 * Errors. Every call returns 0 on success or a negative TT_E* code; tt_strerror names it.
 * Nothing else crosses the ABI (no exceptions). Calls on one stream must not overlap
 * (TT_EBUSY); different streams may be driven from different host threads.
 */
#ifndef TT_H
#define TT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TT_OK 0
#define TT_EINVAL (-1)  /* NULL pointer, bad size, non-finite template, N > M, bad params */
#define TT_ENOMEM (-2)  /* device allocation failed or the stream's HBM budget is exceeded  */
#define TT_ESTATE (-3)  /* frame before template                                           */
#define TT_EDEVICE (-4) /* a HIP call failed, or a device-side bound was hit               */
#define TT_EBUSY (-5)   /* another call is running on the same stream                       */

/* Precision of the normal-equation solve (assembly is FP32 and the LM cost sums FP64 in all forms). */
#define TT_FP32 0    /* FP32 Cholesky: FP32 tile products on the matrix cores, FP32 substitutions        */
#define TT_BF16_IR 1 /* tile products with bfloat16 inputs and FP32 accumulation, then ir_iters steps of
                        iterative refinement whose residual is formed in FP64                             */
#define TT_FP16_IR 2 /* the same with binary16 inputs                                                    */

/* How the damped normal equations of an LM step are solved (tt_params.solver).
 * TT_SOLVE_DENSE: one coupled 6N x 6N system (all ARAP and shared-point couplings), dense
 *   Cholesky; the default.
 * TT_SOLVE_NODE: the literal reading of Sec. 2, where every control point's warp W_i is updated
 *   on its own: only node i's 6 x 6 diagonal block of the damped normal matrix and its part of
 *   J^T r enter node i's step; one Cholesky per node (FP64 on the device), no coupled system.
 *   Only the diagonal blocks are assembled. The LM damping, cost and accept / reject rule are
 *   the same, applied to the step of all nodes together. Ignores precision. */
#define TT_SOLVE_DENSE 0
#define TT_SOLVE_NODE 1

typedef struct tt_stream tt_stream;

typedef struct {
  int width, height;     /* depth map size, >= 3 each */
  double fx, fy, cx, cy; /* pinhole intrinsics in pixels */
} tt_intrinsics;

typedef struct {
  int num_control_points;  /* N >= 1, chosen by farthest-point sampling over the template   */
  int knn;                 /* control points blended per template point; must be 4           */
  double w_orb;            /* weight of f_ORB in Eq. (1); paper: 10                          */
  double w_angle;          /* weight of f_angle in Eq. (5); paper: 20                        */
  double w_rotation;       /* weight of f_rotation in Eq. (5); paper: 100                    */
  double lambda_arap;      /* scale of the dynamic ARAP weight (Sec. 2): 1                   */
  double tukey_c;          /* Tukey constant of f_ICP, mm: 5                                 */
  double H;                /* reweighting threshold of Eq. (4), mm: 3                        */
  int ransac_refs;         /* reference matches per frame (Sec. 2.1): 30                     */
  int ransac_iters;        /* R/w alternations per reference (Sec. 2.1): 10                  */
  int lm_iters;            /* Levenberg-Marquardt iterations per frame: 10                   */
  int max_hamming;         /* matches farther than this are unusable; 256 keeps all          */
  double lm_lambda0;       /* initial Marquardt damping of each frame: 1e-4                  */
  int precision;           /* TT_FP32, TT_BF16_IR or TT_FP16_IR                               */
  uint64_t seed;           /* seed of the reference-match sampler                            */
  uint64_t hbm_budget_bytes; /* 0 = unlimited; otherwise a cap on the stream's device bytes  */
  int ir_iters;            /* refinement steps per solve in the 16-bit forms (0..8); default 2 */
  int solver;              /* TT_SOLVE_DENSE (default) or TT_SOLVE_NODE                        */
  int arap_knn;            /* 0 (default): ARAP over every pair of control points, the dense
                              connection of Sec. 2.2; k in 1..32: only pairs where one node is
                              among the other's k nearest at time 0 (ties to the lower index) */
  int assoc_zbuffer;       /* 0 (default): every deformed template point takes its nearest pixel
                              (Sec. 2's projective association); 1: z-buffered, of the points
                              that project to one pixel only the nearest to the camera (smallest
                              z as float32, ties to the lower index) takes it, the others have no
                              ICP row in that iteration */
  int graph;               /* 0 (default): the LM iterations of each frame are launched kernel by
                              kernel; 1: they are captured once per front-buffer parity into a HIP
                              graph and replayed on later frames (single-stream calls without
                              debug taps or stage timers, and whole-frame batches whose streams
                              all set it; the results are the same bit for bit)               */
  int assoc_kdtree;        /* 0 (default): projective association (Sec. 2's re-projection); 1: the
                              closest-point comparator the paper contrasts it with -- each deformed
                              template point corresponds to the nearest frame point in 3D (float32
                              squared distance, ties to the lower pixel index) among the pixels that
                              have a normal, found through a kd-tree built on the device every frame.
                              Not with assoc_zbuffer. */
} tt_params;

/* Optional per-frame outputs of tt_track_frame; each pointer may be NULL. Sizes: K1 template
 * features, M template points, R = ransac_refs, T = lm_iters, n = 6 N. */
typedef struct {
  int32_t* match_idx;   /* [K1] nearest frame feature by Hamming distance (ties: lower index), -1 if none */
  int32_t* match_dist;  /* [K1] its distance (256 if none) */
  double* wstar;        /* [K1] pre-selection weight: max of w_k over kept hypotheses, 0 if unusable */
  uint8_t* preselected; /* [K1] 1 if w* >= 1/2 */
  int32_t* hyp_k0;      /* [R] reference match of each hypothesis, -1 if fewer usable matches */
  double* hyp_W;        /* [R] sum of w_k after the last reweighting */
  int32_t* hyp_nin;     /* [R] matches with d_k <= H */
  uint8_t* hyp_kept;    /* [R] 1 kept, 0 dropped, 2 degenerate rotation fit */
  int32_t* corr0;       /* [M] iteration-0 pixel of each template point, -1 if none */
  double* r0;           /* [M] iteration-0 point-to-plane residual (0 without a pixel) */
  double* omega0;       /* [M] iteration-0 Tukey weight */
  double* orbw0;        /* [K1] iteration-0 feature weight */
  double* A0;           /* [n*n] iteration-0 J^T J (undamped), row-major, symmetric */
  double* g0;           /* [n] iteration-0 J^T r */
  double* w_arap;       /* [1] dynamic ARAP weight of the frame */
  double* cost_old;     /* [T] cost at the iterate (correspondences of that iteration) */
  double* cost_new;     /* [T] cost at the candidate (NaN if the factorisation failed) */
  double* lambda;       /* [T] damping used */
  uint8_t* accepted;    /* [T] 1 if the candidate was accepted */
  double* delta0;       /* [n] iteration-0 step, node-centred (omega_i, tau_i) per node; unwritten if the factorisation failed */
  double* w_arap_iter;  /* [T] ARAP weight that each iteration's costs and normal equations use */
} tt_frame_debug;

/* Fills every field with the paper's constants and this library's defaults. */
void tt_default_params(tt_params* p);

/* Creates a stream: the state of one tracked surface across the frames of a video (Sec. 2: the
 * template of the first frame and the per-control-point warps carried from frame to frame, each
 * frame's solve starting from the previous warps). p: weights and iteration counts of Eqs. (1)-(6)
 * and Sec. 2.1 (tt_default_params gives the paper's); K: the pinhole camera of the depth maps.
 * hip_stream is a hipStream_t to queue work on (NULL: the library creates its own at default
 * priority) -- an argument the paper has no counterpart for: the caller's queue, so that the
 * solve orders against the caller's own device work without a host round trip. Allocates the
 * frame-size device buffers (the stream owns them; tt_destroy frees them). TT_EINVAL: NULL or
 * out-of-range parameters or intrinsics; TT_ENOMEM / TT_EDEVICE: allocation or stream creation
 * failed (nothing is left allocated). */
int tt_create_stream(const tt_params* p, const tt_intrinsics* K, void* hip_stream, tt_stream** out);

/* Template (Sec. 2, generated from the first frame): pts_xyz [M][3], feat_xyz [K1][3] and
 * feat_desc [K1][32], host memory. Chooses the N control points by farthest-point sampling
 * (start at point 0, ties to the lower index), the 4 nearest control points and Gaussian blend
 * weights of every template point and feature, and the ARAP pair weights; uploads all of it
 * and resets the warps to identity and the frame counter to 0. Synchronous.
 * TT_EINVAL: NULL, M < 1, K1 < 0, N > M, non-finite coordinates, fewer distinct points than N. */
int tt_set_template(tt_stream* s, const float* pts_xyz, int M, const float* feat_xyz,
                    const uint8_t* feat_desc, int K1);

/* One frame from host memory: depth [height][width], feat_xyz [K2][3] (NaN = no depth),
 * feat_desc [K2][32]. Runs the per-frame solve of Sec. 2: the normal map of the depth, Hamming
 * matching of the template's ORB features and their 1-point RANSAC + reweighting pre-selection
 * (Sec. 2.1, Eq. (4)), then lm_iters Levenberg-Marquardt iterations on the cost of Eq. (1)
 * (point-to-plane ICP, ORB and dense ARAP terms, Eqs. (2)-(6)), each a Gauss-Newton system solved
 * by Cholesky factorisation; then writes the deformed template out_vertices [M][3] and the warps
 * out_dq [N][8] (either may be NULL; caller-owned host memory) and the optional debug taps.
 * Synchronous; advances the frame counter. TT_EINVAL: NULL inputs or K2 out of range; TT_ESTATE:
 * no template; TT_EBUSY: another call on the stream; TT_EDEVICE: a HIP call or a device-side
 * check failed. */
int tt_track_frame(tt_stream* s, const float* depth, const float* feat_xyz, const uint8_t* feat_desc,
                   int K2, double* out_vertices, double* out_dq, tt_frame_debug* dbg);

/* Same solve with every array in device memory (d_depth [height][width], d_feat_xyz [K2][3],
 * d_feat_desc [K2][32]; outputs d_out_vertices [M][3] and d_out_dq [N][8] float32, either may
 * be NULL). Queued on the stream's HIP stream and returns without waiting. The inputs must be
 * complete when the call is made, or ordered before the stream's work by the caller (work on
 * another HIP stream, e.g. an upload still in flight, is not waited for; see
 * tt_track_frame_device_ev). */
int tt_track_frame_device(tt_stream* s, const float* d_depth, const float* d_feat_xyz,
                          const uint8_t* d_feat_desc, int K2, float* d_out_vertices, float* d_out_dq);

/* As tt_track_frame_device, except that the frame's inputs count as ready once the HIP event
 * inputs_ready (a hipEvent_t the caller recorded after writing them; NULL: as
 * tt_track_frame_device) has completed, not after all work queued earlier on the stream's HIP
 * stream. The frame's normal map, matching and pre-selection then run on a second HIP stream of
 * the library's while the stream's previous frame is still being solved; its LM iterations start
 * after that frame's, as always. */
int tt_track_frame_device_ev(tt_stream* s, const float* d_depth, const float* d_feat_xyz,
                             const uint8_t* d_feat_desc, int K2, float* d_out_vertices, float* d_out_dq,
                             const void* inputs_ready);

/* One frame for each of several streams, all arrays in device memory (as for
 * tt_track_frame_device). */
typedef struct {
  const float* depth;       /* [height][width] of that stream's intrinsics                     */
  const float* feat_xyz;    /* [K2][3], NaN = no depth                                          */
  const uint8_t* feat_desc; /* [K2][32], 16-byte aligned                                        */
  int K2;
  float* out_vertices;      /* [M][3] float32 or NULL                                           */
  float* out_dq;            /* [N][8] float32 or NULL                                           */
  const void* inputs_ready; /* hipEvent_t after which the inputs are written (as
                               tt_track_frame_device_ev), or NULL                                */
} tt_frame_device;

/* Batched form of tt_track_frame_device: the same per-frame solve (Sec. 2) for S distinct streams
 * (templates, sizes and intrinsics may differ; lm_iters must be equal). The per-stream stages are
 * queued on each stream's own HIP stream; the Cholesky factorisations, substitutions and
 * refinement of all S normal systems run on streams[0]'s HIP stream as one launch each per LM
 * iteration, ordered against the per-stream work by events. The batch starts after all work
 * already queued on every stream's HIP stream, and later work on those HIP streams runs after it
 * (tt_sync on a stream waits for its frame). When every stream sets graph = 1 (and no stage timer
 * is on), the LM set-up and iterations of the batch are captured as one HIP graph per ordered set of
 * streams and pattern of their front-buffer parities, kept until one of its streams is destroyed,
 * gets a new template or new launch shapes, and replayed. Every LM stage of the coupled streams
 * with the default ARAP workgroup, no z-buffer and no stage timer runs as one launch over all of
 * them on streams[0]'s HIP stream, over a small device table of their arguments (kept with the
 * graph, or written per call into a ring of four slots held by streams[0]); the other streams'
 * stages run as their own launches. Each stream's result is the same as when it is tracked alone. Returns without waiting. TT_EINVAL: bad arguments or a stream listed twice;
 * TT_EBUSY: a stream is in use by another call (no stream is then touched); TT_ESTATE: a stream
 * has no template. */
int tt_track_batch_device(tt_stream* const* streams, int S, const tt_frame_device* frames);

/* Waits for the stream's queued work; returns TT_EDEVICE if a device-side check failed. */
int tt_sync(tt_stream* s);

/* The LM record of the stream's last frame (Sec. 2: one Levenberg-Marquardt step per iteration),
 * each array [lm_iters] or NULL: the cost at the iterate and at the candidate (NaN where the
 * factorisation failed), the damping, 1 where the candidate was accepted, the ARAP weight of each
 * iteration, 1 where the factorisation failed. Waits for the stream's queued work first. */
int tt_get_frame_log(tt_stream* s, double* cost_old, double* cost_new, double* lambda, uint8_t* accepted,
                     double* w_arap, int32_t* chol_fail);

/* The hipStream_t the stream queues on. */
void* tt_hip_stream(tt_stream* s);

/* Template queries: node_idx [N], knn_pts [M][4], alpha_pts [M][4], knn_feat [K1][4],
 * alpha_feat [K1][4], sbar and s_arap (scalars); any may be NULL. */
int tt_get_template_info(tt_stream* s, int32_t* node_idx, int32_t* knn_pts, float* alpha_pts,
                         int32_t* knn_feat, float* alpha_feat, double* sbar, double* s_arap);

/* Warp state (N x 8, double on the host) and frame counter: read, or set for teacher forcing. */
int tt_get_state(tt_stream* s, double* dq, int64_t* frame);
int tt_set_state(tt_stream* s, const double* dq, int64_t frame);

/* Per-stage GPU timers (hipEvents recorded on the stream's HIP stream around each stage). */
#define TT_STAGE_FRONT 0  /* normal map, Hamming matching, 1-point RANSAC pre-selection */
#define TT_STAGE_ROWS 1   /* per-point / per-feature residual and Jacobian rows          */
#define TT_STAGE_ARAP 2   /* dense ARAP assembly into the normal matrix                  */
#define TT_STAGE_DATA 3   /* data-term block assembly (block-CSR)                        */
#define TT_STAGE_SOLVE 4  /* damping and equilibration, back substitution               */
#define TT_STAGE_UPDATE 5 /* candidate warps, FP64 costs, accept / reject               */
#define TT_STAGE_FACTOR 6 /* blocked Cholesky factorisation with the forward substitution */
#define TT_NSTAGES 7

#define TT_TIMING_ALL ((1 << TT_NSTAGES) - 1)

/* Selects the stages whose GPU time is measured: bit i of stages (0 <= stages <= TT_TIMING_ALL)
 * times stage i, 0 turns the timers off. Each timed stage records two HIP events on the stream
 * per call, so time only what is needed where the throughput itself is measured. Untimed, the
 * rows and the ARAP assembly of every LM iteration after the first run as one launch; timing
 * either of the two stages keeps them as two launches (same results, each between its own events).
 * TT_EINVAL for a bit outside the stages. */
int tt_set_timing(tt_stream* s, int stages);

/* Waits for the stream, then returns the GPU milliseconds accumulated per stage since the last
 * call (ms [TT_NSTAGES]) and how many times each stage ran (count [TT_NSTAGES]); either may be
 * NULL. Resets the accumulators. */
int tt_get_timing(tt_stream* s, double* ms, int64_t* count);

/* Diagnostic: solves A x = b with the library's dense FP32 Cholesky path (the same kernels as the
 * LM step: blocked factorisation with the right-hand side carried along, then back substitution).
 * A is n x n row-major (symmetric; the lower triangle is read), b and x have n entries, host
 * memory. *fail receives 1 if a pivot was not positive. Allocates and frees its own device
 * memory; synchronous. */
int tt_debug_cholesky_solve(int n, const float* A, const float* b, float* x, int* fail);

/* The same with a precision form (TT_FP32, TT_BF16_IR, TT_FP16_IR) and ir_iters refinement steps
 * (ignored for TT_FP32): the diagnostic of the 16-bit solve and its refinement. */
int tt_debug_cholesky_solve_ex(int n, const float* A, const float* b, float* x, int* fail, int precision,
                               int ir_iters);

/* Device bytes held by the stream. */
int tt_device_bytes(tt_stream* s, uint64_t* bytes);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops): the FP32 form of tt_debug_cholesky_solve_ex on device buffers, allocating nothing. Every
 * workspace (padded working matrix, inverse diagonal blocks, hand-over flags, scalars, scaling,
 * solution) lives in one static device array of TT_NOALLOC_SCRATCH_BYTES that each GPU the library
 * runs on holds until the process ends; the first call on a GPU resolves its address once.
 * d_A [n][n] row-major, SPD, lower triangle read; d_b [n]; d_x [n] receives x; d_status [2]
 * receives (1 if a pivot was not positive, device error bits). All device memory, caller-owned.
 * Queued on hip_stream (a hipStream_t; NULL: the null stream), returns without waiting.
 * TT_EINVAL: n outside 1..TT_NOALLOC_MAX_N or a NULL buffer. Calls on one GPU share the array, which
 * keeps the last call's contents: calls that overlap on one GPU race (queue them on one stream). */
#define TT_NOALLOC_MAX_N 1024
#define TT_NOALLOC_SCRATCH_BYTES 4736768
int tt_cholesky_solve_noalloc(int n, const float* d_A, const float* d_b, float* d_x, int32_t* d_status,
                              void* hip_stream);

/* ---- Tuning ------------------------------------------------------------------------------
 * Launch shapes of the per-frame solve that do not change what it computes: the width of the
 * factorisation's persistent launch, the size of the dense-ARAP workgroups and whether the rows
 * and ARAP kernels share one launch after the first LM iteration. The factorisation and the fusion
 * leave every result bit for bit the same; the ARAP workgroup size changes the order in which a
 * node's diagonal block and gradient terms are summed (FP32 rounding only). */
typedef struct {
  int chol_grid_pct;  /* workgroups of the factorisation launch, in percent of the compute units
                         (25..400; default 200; at most one workgroup per task); a batched
                         launch takes the largest of its systems' values                       */
  int arap_threads;   /* 128 or 256 (default) threads per dense-ARAP workgroup                   */
  int fuse_rows_arap; /* 1 (default): rows and ARAP in one launch from the second LM iteration on
                         (needs arap_threads 256); 0: separate launches                          */
  double frame_ms;    /* tt_autotune: mean time per frame of this configuration, else 0          */
} tt_tuning;
int tt_get_tuning(tt_stream* s, tt_tuning* out);
/* TT_EINVAL: a field out of range. Captured LM graphs are dropped and recaptured with the new shapes. */
int tt_set_tuning(tt_stream* s, const tt_tuning* t);
/* Project-written autotuner: times the whole per-frame solve of one of the caller's frames (device
 * arrays as tt_track_frame_device) under each candidate -- launch width 50 / 100 / 200 % x (ARAP
 * 256 fused, 256 unfused, 128 unfused) -- one untimed and reps timed frames each (1..100), every
 * frame starting from the stream's warps and frame counter as they were, which are restored
 * afterwards; keeps the fastest, returns it in *best with its time. Synchronous. TT_ESTATE: no
 * template. */
int tt_autotune(tt_stream* s, const float* d_depth, const float* d_feat_xyz, const uint8_t* d_feat_desc, int K2,
                int reps, tt_tuning* best);

/* Destroys the stream (the surface of Sec. 2 it tracked: template, warps, frame buffers) after its
 * queued work has finished, and frees its device memory and, if the library created it, its HIP
 * stream. TT_EINVAL: NULL; TT_EBUSY: a server owns the stream (tt_server_close destroys it). */
int tt_destroy(tt_stream* s);

/* ---- Serving: many streams under one HBM budget, continuous batching ----------------------
 * The per-frame solve of Sec. 2 for many independent streams at once. A server owns the streams it
 * opens (other calls on them return TT_EBUSY until tt_server_close) and runs one scheduler thread
 * that queues the streams' work in rounds of one LM iteration: in a round every frame in flight
 * assembles its normal system, all those systems are factored and solved together (one batched
 * launch per up to 32 systems, on the server's HIP stream), and every frame takes its update. The
 * frames of coupled streams with no stage of their own (no per-node solve, z-buffer, 128-thread
 * ARAP workgroups or stage timers) run every stage of the round on the server's HIP stream as one
 * launch over all of them; the others assemble and update on their stream's HIP stream. A submitted frame first has its normal map, matching and pre-selection queued on
 * its stream's side queue; it joins the rounds at the first LM-iteration boundary after that stage
 * has finished, and leaves after its lm_iters-th iteration, so frames of different streams enter
 * and leave at iteration boundaries rather than in whole-frame batches. Frames of one stream run in
 * submission order. Each frame's result is the same as when its stream is tracked alone.
 *
 * Admission: every open stream holds its device bytes (tt_device_bytes, with the feature buffers
 * sized for K2max at open) against the server's hbm_budget_bytes. An open that does not fit waits,
 * in arrival order, until tt_server_close releases enough bytes or wait_s runs out (TT_EBUSY); one
 * that could not fit even in an empty server returns TT_ENOMEM.
 * Latency: from tt_server_submit to the moment the scheduler sees the frame's last kernel complete
 * (front stage included), on the host's steady clock. */
typedef struct tt_server tt_server;
typedef struct {
  uint64_t hbm_budget_bytes; /* device bytes all open streams may hold together; 0 = unlimited   */
  int max_rounds_ahead;      /* rounds queued ahead of the device (1..8; 0 = the default, 1): a new
                                frame joins after at most this many rounds already queued; more
                                run-ahead only makes the rounds smaller (measured at config 4)     */
} tt_server_params;

typedef struct {
  int streams_open;          /* admitted streams                                                  */
  int opens_waiting;         /* tt_server_open calls waiting for budget                           */
  uint64_t reserved_bytes;   /* device bytes held by the open streams                             */
  int64_t frames_submitted;
  int64_t frames_done;
  int64_t rounds;            /* LM-iteration rounds queued                                        */
  int64_t frame_iterations;  /* sum over rounds of the frames in that round                       */
} tt_server_stats;

void tt_server_default_params(tt_server_params* p);
/* hip_stream: the HIP stream the batched solves run on (NULL: the server creates one). The device
 * current at this call is the one the scheduler thread uses. */
int tt_server_create(const tt_server_params* p, void* hip_stream, tt_server** out);
/* tt_create_stream + tt_set_template under the budget (arguments as there; K2max: the most
 * features any frame of this stream will have). On success *out is open and owned by the server. */
int tt_server_open(tt_server* sv, const tt_params* p, const tt_intrinsics* K, const float* pts_xyz, int M,
                   const float* feat_xyz, const uint8_t* feat_desc, int K1, int K2max, double wait_s,
                   tt_stream** out);
/* Queues one frame of an open stream (device arrays as tt_frame_device; they must stay unchanged
 * until the frame is reported done; K2 <= K2max). *ticket identifies it for tt_server_poll/_wait.
 * Returns at once. TT_EINVAL: bad arguments or a stream this server does not own. */
int tt_server_submit(tt_server* sv, tt_stream* s, const tt_frame_device* f, uint64_t* ticket);
/* *done = 1 once the frame's outputs are written; its latency (ms) in *latency_ms, and the return
 * value is the frame's status (TT_EDEVICE if a device-side check failed). A ticket is forgotten once
 * reported done. TT_EINVAL: unknown ticket. */
int tt_server_poll(tt_server* sv, uint64_t ticket, int* done, double* latency_ms);
/* As tt_server_poll, blocking until done or wait_s has passed (then TT_EBUSY). */
int tt_server_wait(tt_server* sv, uint64_t ticket, double wait_s, double* latency_ms);
/* Waits for the stream's frames, destroys it and releases its bytes to waiting opens. */
int tt_server_close(tt_server* sv, tt_stream* s);
int tt_server_get_stats(tt_server* sv, tt_server_stats* out);
/* Waits for every frame, closes every open stream, stops the scheduler. */
int tt_server_destroy(tt_server* sv);

const char* tt_strerror(int code);

/* ---- Uniform ORB features (Sec. 2.1) ------------------------------------------------------
 * The paper detects FAST corners for every pixel in parallel on the GPU and suppresses a corner
 * when a neighbouring pixel has a larger corner response, so that features spread over low-
 * texture areas too, then describes them as ORB features. Definitions (all integer except the
 * orientation bin, which is taken in FP64 from integer moments):
 *   corner    FAST-9: of the 16 pixels of the radius-3 circle, 9 or more contiguous (cyclic) are
 *             all brighter than I_p + t or all darker than I_p - t; response = max(sum over the
 *             brighter of (I - I_p - t), sum over the darker of (I_p - I - t)), else 0;
 *   region    pixels at least TT_ORB_BORDER from every image border;
 *   kept      no other corner in the (2r+1)^2 window has a larger response (ties: the lower
 *             pixel index wins); keypoints in raster order, at most max_features of them;
 *   angle     intensity centroid atan2(m01, m10) over the disc of radius 15, in 30 bins of 12
 *             degrees, rounded to the nearest bin;
 *   desc      256 tests on the 5x5 box sums S of the image: bit k (byte k / 8, bit k % 8 from
 *             the least significant) = S(p + a_k) < S(p + b_k), (a_k, b_k) = pattern row k =
 *             (x1, y1, x2, y2) rotated by the angle bin and rounded half away from zero;
 *   xyz       the back-projection of the depth at the keypoint (NaN when invalid or no depth).
 * These descriptors and points are what tt_set_template / tt_track_frame take as features. */
#define TT_ORB_BORDER 18

typedef struct tt_orb tt_orb;

typedef struct {
  int fast_threshold; /* t, 0..255; default 20 */
  int nms_radius;     /* r, 0..16; default 1 (the 8 neighbouring pixels) */
  int max_features;   /* cap on keypoints, 0..2^20; default 4096 */
} tt_orb_params;

void tt_orb_default_params(tt_orb_params* p);

/* A detector for width x height 8-bit images. pattern: [256][4] int8 host array of point
 * pairs (x1, y1, x2, y2), each point within radius 13 of the keypoint (TT_EINVAL otherwise);
 * copied. hip_stream: a hipStream_t for the work (NULL: the detector creates its own). */
int tt_orb_create(const tt_orb_params* p, int width, int height, const int8_t* pattern, void* hip_stream,
                  tt_orb** out);

/* Device-memory detection, queued on the detector's HIP stream (returns without waiting).
 * d_image [height][width] uint8; d_depth [height][width] float32 or NULL (then K may be NULL);
 * outputs d_kp [max][2] int32 (u, v), d_desc [max][32], d_xyz [max][3] float32 (or NULL),
 * d_angle [max] int32 bins (or NULL), d_count [2] int32: keypoints written, corners kept before
 * the cap. Entries past d_count[0] are left as they were. */
int tt_orb_detect_device(tt_orb* o, const uint8_t* d_image, const float* d_depth, const tt_intrinsics* K,
                         int32_t* d_kp, float* d_xyz, uint8_t* d_desc, int32_t* d_angle, int32_t* d_count);

/* The same from and to host memory (outputs sized for max_features), synchronous. */
int tt_orb_detect(tt_orb* o, const uint8_t* image, const float* depth, const tt_intrinsics* K, int32_t* kp,
                  float* xyz, uint8_t* desc, int32_t* angle, int32_t* count);

/* Calls on one detector must not overlap (TT_EBUSY); different detectors may be used from
 * different host threads. */

/* The detector's hipStream_t. */
void* tt_orb_hip_stream(tt_orb* o);

int tt_orb_destroy(tt_orb* o);

#ifdef __cplusplus
}
#endif

#endif
