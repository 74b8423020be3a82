// tt_internal.h -- device-side state of one tracked stream and the kernel launchers.
//
// Data layout in HBM (all resident for the life of the stream unless marked per frame):
//   template points   px, py, pz          f32 [M]        (SoA, coalesced per point)
//                     knn                 int4 [M]       (4 nearest control points)
//                     alpha               float4 [M]     (Gaussian blend weights)
//   template features fpx, fpy, fpz       f32 [K1]; fknn int4 [K1]; falpha float4 [K1]
//                     desc                uint32 [8][K1] (256-bit descriptors as 8 word planes)
//   control points    c0                  float4 [N]     (rest position p_i^0)
//                     W, Wc               f32 [N][8]     (current / candidate dual quaternion)
//                     pos                 float4 [N]     (p_i^t of the current warps)
//   data-term blocks  blk_ab, blk_ptr, blk_ent: static block-CSR of node pairs (a >= b) that
//                     share a template point or feature, with the contributing rows
//   per frame         depth f32 [H*W]; nmap float4 [H*W] = (n, z) of the target surface
//   per iteration     jac f32 [M][24], wres f32 [M] (weighted ICP rows); jacF f32 [K1][72],
//                     wresF f32 [3][K1] (weighted feature rows); the Jacobian rows are per point so
//                     that the block assembly reads each point's 2 x 6 entries as contiguous pairs
//   normal matrix     A f32 [(npad + 64) x npad] row-major, lower triangle; rows npad..npad+63
//                     hold the right-hand side row(s) so that the forward substitution runs
//                     inside the blocked factorisation; Linv f32 [nb][64][64] inverse diagonal
//                     blocks for the back substitution.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <mutex>
#include <vector>

#include "../../include/tt.h"

#define TT_NB 64  // Cholesky block size

struct LMScalars {
  double lambda;     // Marquardt damping of the current iteration
  double e_old;      // cost at the iterate
  double e_new;      // cost at the candidate
  double w_arap;     // dynamic ARAP weight of the frame
  double sum_omega;  // sum of Tukey weights (iteration 0)
  double sum_orbw;   // sum of feature weights (iteration 0)
  double eps;        // diagonal shift of the damping
  int chol_fail;     // set by the factorisation when a pivot is not positive
  int accept;        // decision of the last iteration
  int it;            // iteration counter
  int err;           // device-side error bits (TT_DEVERR_*), reported as TT_EDEVICE
  int solve_epoch;   // epoch of the current solve (set by the damping kernel)
};

#define TT_DEVERR_CHOL_SYNC 1  // a hand-over wait of the factorisation passed its deadline

struct DevState {
  // sizes
  int M = 0, N = 0, K1 = 0, HW = 0, n = 0, npad = 0, nb = 0, ld = 0;
  int K2cap = 0;
  // template
  float *px = nullptr, *py = nullptr, *pz = nullptr;
  int4* knn = nullptr;
  float4* alpha = nullptr;
  float *fpx = nullptr, *fpy = nullptr, *fpz = nullptr;
  int4* fknn = nullptr;
  float4* falpha = nullptr;
  uint32_t* desc = nullptr;
  float4* c0 = nullptr;
  int* node_idx = nullptr;
  double* mind = nullptr;  // FPS scratch [M]
  int nblk = 0;
  int2* blk_ab = nullptr;
  int* blk_ptr = nullptr;
  uint32_t* blk_ent = nullptr;
  double sbar = 0.0, s_arap = 0.0;
  uint32_t* adj = nullptr;   // [N][adj_words] sparse ARAP graph bit rows (nullptr: every pair)
  int adj_words = 0;
  unsigned long long* zbuf = nullptr; // [HW] z-buffer keys (z bits << 32 | point), z-buffered association
  int* zpix = nullptr;       // [M] pixel of each deformed template point in the z-buffer pass
  // warps
  float *W = nullptr, *Wc = nullptr;
  float4 *pos = nullptr, *posc = nullptr;    // p_i^t
  float4 *ndisp = nullptr, *ndispc = nullptr;  // p_i^t - p_i^0
  // frame inputs (staging)
  float* depth = nullptr;
  float4* nmap = nullptr;    // the current frame's set of the double-buffered front outputs
  // Front outputs the LM iterations read (nmap, o2, wstar, presel) come in two sets, so that the
  // next frame's front stage can fill one while the current frame's iterations read the other;
  // set f starts at base + f * count.
  float4* nmap_b = nullptr;
  float4* o2_b = nullptr;
  double* wstar_b = nullptr;
  uint8_t* presel_b = nullptr;
  size_t K1a = 0;
  float* f2xyz = nullptr;    // [K2cap][3]
  uint32_t* f2desc = nullptr;  // [8][K2cap]
  // matching + pre-selection
  int* midx = nullptr;
  int* mdist = nullptr;
  float4* o2 = nullptr;      // [K1] matched frame point, w = 1 if usable
  int* ulist = nullptr;      // [K1] usable list / shuffle workspace
  int* refs = nullptr;       // [R]
  double* hyp_w = nullptr;   // [R][K1]
  double* hyp_W = nullptr;   // [R]
  int* hyp_nin = nullptr;    // [R]
  int* hyp_state = nullptr;  // [R] 1 kept, 0 dropped, 2 degenerate, -1 not drawn
  double* wstar = nullptr;   // [K1]
  uint8_t* presel = nullptr; // [K1]
  // LM
  int* corr = nullptr;
  float* rres = nullptr;
  float* omega = nullptr;
  float* jac = nullptr;      // [M][24]
  float* wres = nullptr;     // [M]
  float* orbw = nullptr;     // [K1]
  float* jacF = nullptr;     // [K1][72]
  float* wresF = nullptr;    // [3][K1]
  float* A = nullptr;        // [(npad + TT_NB) * ld]
  float* g = nullptr;        // [npad]
  float* x = nullptr;        // [npad] solution of the equilibrated system
  float* dscale = nullptr;   // [npad] symmetric diagonal equilibration d_k = 1/sqrt(damped A_kk)
  float* Linv = nullptr;     // [nb][TT_NB][TT_NB]
  int* flags = nullptr;      // [chol_flag_ints(nb)] factorisation and back-substitution flags
  int num_cus = 0;           // compute units of the device (persistent launch size)
  int wall_khz = 0;          // rate of the device's constant clock (s_memrealtime), kHz
  // tuning (tt_set_tuning / tt_autotune): width of the factorisation launch in percent of the compute
  // units, threads per dense-ARAP workgroup, and whether rows and ARAP share a launch after iteration 0
  int chol_grid_pct = 200;
  // kd-tree association (assoc_kdtree): per front-buffer set the frame's points in tree order, the
  // split values (heap order) and the point count; build scratch (tt_kdtree.hip)
  float4* kd_pts_b = nullptr;
  float* kd_split_b = nullptr;
  int* kd_count_b = nullptr;
  float4* kd_pts = nullptr;
  float* kd_split = nullptr;
  int* kd_count = nullptr;
  int kd_levels = 0;
  uint8_t* kd_flag = nullptr;
  int* kd_sel = nullptr;
  float4* kd_xyz = nullptr;
  uint32_t* kd_vals = nullptr;  // [2][HW]
  uint64_t* kd_keys = nullptr;  // [2][HW]
  void* kd_temp = nullptr;
  size_t kd_temp_bytes = 0;
  int arap_threads = 256;
  int fuse_rows_arap = 1;
  int prec = TT_FP32;        // precision form of the solve
  int ir_iters = 0;          // refinement steps per solve (16-bit forms)
  int solver = TT_SOLVE_DENSE; // coupled dense solve or one 6 x 6 solve per node
  uint16_t* A16 = nullptr;   // 16-bit copies of the finished L tiles [(npad + 64) * ld]
  float* A0 = nullptr;       // damped matrix before factorisation [npad * ld] (refinement)
  float* cvec = nullptr;     // equilibrated right-hand side [npad] (refinement)
  double* xd = nullptr;      // FP64 solution of the refinement [npad], then the residual's partial sums
                             // [nb * nb * 64] (ir_xd_count)
  uint64_t* tw = nullptr;    // [npad] tagged entries (epoch << 32 | float) of a running substitution
  double* partial = nullptr; // reduction partials
  int npartial = 0;
  LMScalars* sc = nullptr;
  double* log_cost_old = nullptr;
  double* log_cost_new = nullptr;
  double* log_lambda = nullptr;
  int* log_accept = nullptr;
  double* log_w_arap = nullptr;   // [T] ARAP weight used by each iteration of the last frame
  int* log_fail = nullptr;        // [T] 1 where the iteration's factorisation failed
  // debug copies
  float* A_dbg = nullptr;
  float* g_dbg = nullptr;
  int* corr_dbg = nullptr;
  float* rres_dbg = nullptr;
  float* omega_dbg = nullptr;
  float* orbw_dbg = nullptr;
  float* x_dbg = nullptr;     // iteration-0 solution and equilibration [2 npad]
};

struct tt_stream {
  tt_params P;
  tt_intrinsics K;
  hipStream_t st = nullptr;
  bool own_stream = false;
  bool has_template = false;
  int64_t frame = 0;
  std::mutex mu;
  std::atomic<bool> served{false};  // owned by a tt_server: the stream's own entry points return TT_EBUSY
  DevState d;
  std::vector<void*> allocs_template;  // freed on re-template / destroy
  std::vector<void*> allocs_frame;     // frame-size buffers (created with the stream)
  std::vector<void*> allocs_k2;        // grows with K2
  uint64_t bytes_template = 0, bytes_frame = 0, bytes_k2 = 0;
  // stage timers
  unsigned timing = 0;  // bit i set: stage i is timed
  std::vector<hipEvent_t> ev_pool;       // timing events
  std::vector<hipEvent_t> ev_sync_pool;  // ordering events between HIP streams (batched path)
  // argument tables of the multi-system launches of the batches this stream leads (streams[0])
  // that are not graph-replayed: a ring of pinned staging slots, their device copies (written on
  // this stream's HIP stream, behind every earlier batch that reads them) and an event after each
  // slot's copy, waited on before the slot is written again
  std::vector<void*> bt_host, bt_dev;
  std::vector<hipEvent_t> bt_ev;
  size_t bt_cap = 0, bt_next = 0;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
  double stage_ms[TT_NSTAGES] = {};
  int64_t stage_n[TT_NSTAGES] = {};
  // the front stage (normal map, matching, pre-selection) of a frame runs on its own HIP stream,
  // overlapping the previous frame's LM iterations; per buffer set f: front done / LM done
  hipStream_t st_front = nullptr;
  hipEvent_t ev_front_done[2] = {nullptr, nullptr};
  hipEvent_t ev_lm_done[2] = {nullptr, nullptr};
  // graph mode: the frame's LM iterations captured once per front-buffer set (they read only the
  // stream's own buffers, so a replay does the same work on the next frame of that parity)
  hipGraphExec_t lm_graph[2] = {nullptr, nullptr};
};

// Points d's front outputs at buffer set f (0 or 1).
inline void select_front_set(DevState& d, int f) {
  d.nmap = d.nmap_b + (size_t)f * d.HW;
  if (d.kd_pts_b) {
    d.kd_pts = d.kd_pts_b + (size_t)f * d.HW;
    d.kd_split = d.kd_split_b + ((size_t)f << d.kd_levels);
    d.kd_count = d.kd_count_b + f;
  }
  if (d.o2_b) {
    d.o2 = d.o2_b + (size_t)f * d.K1a;
    d.wstar = d.wstar_b + (size_t)f * d.K1a;
    d.presel = d.presel_b + (size_t)f * d.K1a;
  }
}

// ---- launchers (each queues kernels on st and returns hipGetLastError()) --------------------
struct Intr {
  int W, H;
  double fx, fy, cx, cy;
};

hipError_t launch_fps(const DevState& d, int M, int N, int* err_flag, hipStream_t st);
hipError_t launch_template_tables(DevState& d, hipStream_t st, double* sbar_out, double* sarap_out);
hipError_t launch_node_graph(DevState& d, int k, hipStream_t st);
hipError_t launch_knn(const DevState& d, double sbar, hipStream_t st);

hipError_t launch_normal_map(const DevState& d, const Intr& K, hipStream_t st);
// kd-tree of the frame's points (assoc_kdtree), into the current front-buffer set
constexpr int kKdLeaf = 16;  // most points in a leaf
int kd_levels_for(int HW);
size_t kd_scratch_bytes(int HW);
hipError_t launch_kd_build(DevState& d, const Intr& K, hipStream_t st);
hipError_t launch_match(const DevState& d, int K2, int max_hamming, hipStream_t st);
hipError_t launch_preselect(const DevState& d, int R, int iters, double H, uint64_t seed, int64_t frame,
                            hipStream_t st);

hipError_t launch_lm_begin(DevState& d, double lambda0, hipStream_t st);
hipError_t launch_lm_rows(DevState& d, const tt_params& P, const Intr& K, int it, hipStream_t st);
hipError_t launch_lm_arap(DevState& d, const tt_params& P, hipStream_t st);
// Rows and dense ARAP blocks in one launch; iterations after the first only (the ARAP weight is set
// by iteration 0's rows).
hipError_t launch_lm_rows_arap(DevState& d, const tt_params& P, const Intr& K, int it, hipStream_t st);
hipError_t launch_lm_data(DevState& d, hipStream_t st);
hipError_t launch_lm_damp(DevState& d, hipStream_t st);
hipError_t launch_node_solve(DevState& d, hipStream_t st);
hipError_t launch_lm_finish(DevState& d, const tt_params& P, const Intr& K, hipStream_t st);
hipError_t launch_deform_out(const DevState& d, float* out_xyz, float* out_dq, hipStream_t st);

// Multi-system LM launches: the per-iteration stages of several coupled systems (no per-node solve,
// no z-buffer) as one launch each, over a device table of their arguments (built from frame views,
// so one table per batch composition and front-buffer parity). Each system's results are bit for
// bit those of its own launches.
struct LMMulti {
  void* jobs = nullptr;  // device table, one entry per system
  int nj = 0;
  int blocks[5] = {};    // workgroups of the node-shaped, row-shaped, data-block, row-block and ARAP grids
};
// Synchronous (allocates and copies the table); hipErrorInvalidValue for a system it does not cover.
hipError_t lm_multi_build(DevState* const* ds, const tt_params* const* P, const Intr* K, int S, LMMulti* out);
// Bytes of a table of S systems.
size_t lm_multi_bytes(int S);
// Writes the table into host memory (lm_multi_bytes(S) bytes) and describes it as living at dev;
// the caller copies host to dev before the launches read it.
hipError_t lm_multi_fill(DevState* const* ds, const tt_params* const* P, const Intr* K, int S, void* host,
                         void* dev, LMMulti* out);
void lm_multi_free(LMMulti& m);
// LM set-up of every system (launch_lm_begin)
hipError_t launch_lm_multi_begin(const LMMulti& m, hipStream_t st);
// rows and dense ARAP (at iteration 0: rows, ARAP weight, ARAP blocks), data blocks, damping of
// every system
hipError_t launch_lm_multi_assemble(const LMMulti& m, int it, hipStream_t st);
// candidate, FP64 cost, accept / reject of every system
hipError_t launch_lm_multi_finish(const LMMulti& m, hipStream_t st);

// Ints of the flag area used by one Cholesky solve (tile flags, ticket counters, abort word).
size_t chol_flag_ints(int nb);
// Factorisation of the damped, equilibrated system (forward substitution included), then the back
// substitution into d.x. The solve's flags carry the epoch in d.sc->solve_epoch (set on the device
// by the damping kernel), so a launch's arguments stay the same from one solve to the next; `which`
// numbers a substitution launch within the solve (0: the back substitution after the factorisation).
hipError_t launch_cholesky_factor(DevState& d, hipStream_t st);
hipError_t launch_cholesky_backsolve(DevState& d, int which, hipStream_t st);
// The same for S independent systems at once (one launch per 32 systems).
hipError_t launch_cholesky_factor_batch(DevState* const* ds, int S, hipStream_t st);
hipError_t launch_cholesky_backsolve_batch(DevState* const* ds, int which, int S, hipStream_t st);
// Refinement (16-bit forms): keep the damped matrix and right-hand side before the factorisation;
// xd = x (mode 0) or xd += x, x = xd (mode 1); refinement step `step` (0, 1, ...) = FP64 residual,
// forward and back substitution, accumulation.
// doubles of the refinement's xd buffer: the solution and the residual's per-tile partial sums
inline size_t ir_xd_count(int npad, int nb) { return (size_t)npad + (size_t)nb * nb * TT_NB; }
hipError_t launch_ir_prepare(DevState& d, hipStream_t st);
hipError_t launch_ir_prepare_batch(DevState* const* ds, int S, hipStream_t st);
hipError_t launch_ir_accum_batch(DevState* const* ds, int S, int mode, hipStream_t st);
hipError_t launch_ir_step_batch(DevState* const* ds, int step, int S, hipStream_t st);

// ---- per-frame queueing steps, shared with the serving loop (defined in tt_api.hip) -----------
// The same steps the single-stream and batched paths queue, in the same order: front (normal map,
// matching, pre-selection on the stream's side queue), LM set-up, per iteration assemble -> solve
// (batched over systems) -> finish, then the deformed outputs. The caller holds the stream's lock.
namespace ttx {
DevState frame_view(tt_stream* s, const float* depth, const float* xyz, const uint8_t* desc);
int ensure_k2(tt_stream* s, int K2);
int enqueue_front(tt_stream* s, DevState& dd, int K2, hipStream_t st, const void* inputs_ready);
hipEvent_t front_done_event(tt_stream* s);  // the event enqueue_front recorded for the stream's current frame
bool multi_ok(const tt_stream* s);          // LM stages may run as multi-system launches
Intr intr(const tt_stream* s);
int enqueue_lm_begin(tt_stream* s, hipStream_t st);
int enqueue_assemble(tt_stream* s, DevState& dd, int it, hipStream_t st);
int enqueue_solve(tt_stream* const* ss, DevState* const* dp, int S, hipStream_t st);
int enqueue_node_solve(tt_stream* s, DevState& dd, hipStream_t st);
int enqueue_finish(tt_stream* s, DevState& dd, hipStream_t st);
// deformed outputs, the frame's buffer set released, frame counter advanced
int enqueue_frame_end(tt_stream* s, float* out_xyz, float* out_dq, hipStream_t st);
hipError_t ev_sync_get(tt_stream* s, hipEvent_t* e);
void ev_sync_put(tt_stream* s, hipEvent_t e);
}  // namespace ttx
