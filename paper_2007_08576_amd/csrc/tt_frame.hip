// tt_frame.hip -- template set-up and per-frame front kernels for gfx950:
//   * control points by farthest-point sampling, blend neighbours and Gaussian weights
//     (Sec. 2: sparse control points whose warps the template interpolates); the optional
//     k-nearest-node ARAP graph (the sparse alternative to Sec. 2.2's dense connection);
//   * target normal map from the depth map (Sec. 2: point-to-plane ICP along the normal);
//   * Hamming matching of template ORB descriptors against the frame (Sec. 2.1);
//   * 1-point RANSAC + reweighting inlier pre-selection in FP64 (Sec. 2.1, Eqs. (2)-(4)).
//
// Every decision that selects an index (farthest point, nearest nodes, nearest descriptor,
// pre-selected set) is taken in a precision and operation order that do not depend on the
// launch shape: squared distances in FP64 with no FMA contraction, integer keys for argmin.
#include <float.h>

#include "tt_internal.h"
#include "tt_math.h"

namespace {

constexpr int kWave = 64;

// (value, index) argmax with ties to the lower index
struct VI {
  double v;
  int i;
};
__device__ __forceinline__ VI vi_better(VI a, VI b) {
  if (b.v > a.v || (b.v == a.v && b.i < a.i && b.i >= 0)) return b;
  return a;
}

// squared distance in FP64 from float coordinates, dx*dx + dy*dy + dz*dz left to right
__device__ __forceinline__ double d2_f64(float ax, float ay, float az, float bx, float by, float bz) {
#pragma clang fp contract(off)
  double dx = (double)ax - (double)bx;
  double dy = (double)ay - (double)by;
  double dz = (double)az - (double)bz;
  return dx * dx + dy * dy + dz * dz;
}

template <int BS>
__device__ double block_sum_d(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int s = BS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------------------------------------
// Farthest-point sampling: one workgroup walks the N selections; each step refreshes every
// point's squared distance to the chosen set and takes the farthest, lowest index on ties.

constexpr int kFpsThreads = 1024;

__global__ __launch_bounds__(kFpsThreads) void k_fps(const float* __restrict__ px, const float* __restrict__ py,
                                                     const float* __restrict__ pz, int M, int N,
                                                     double* __restrict__ mind, int* __restrict__ node_idx,
                                                     float4* __restrict__ c0, int* __restrict__ err) {
  __shared__ double sv[kFpsThreads];
  __shared__ int si[kFpsThreads];
  __shared__ int cur;
  __shared__ int bad;
  const int tid = threadIdx.x;
  for (int j = tid; j < M; j += kFpsThreads) mind[j] = DBL_MAX;
  if (tid == 0) {
    cur = 0;
    bad = 0;
  }
  __syncthreads();
  for (int i = 0; i < N; i++) {
    const int c = cur;
    if (tid == 0) {
      node_idx[i] = c;
      c0[i] = make_float4(px[c], py[c], pz[c], 0.0f);
    }
    if (i == N - 1) break;
    const float cx = px[c], cy = py[c], cz = pz[c];
    VI best{-1.0, -1};
    for (int j = tid; j < M; j += kFpsThreads) {
      double d = d2_f64(px[j], py[j], pz[j], cx, cy, cz);
      double m = mind[j];
      if (d < m) {
        m = d;
        mind[j] = m;
      }
      if (m > best.v) best = VI{m, j};
    }
    sv[tid] = best.v;
    si[tid] = best.i;
    __syncthreads();
    for (int s = kFpsThreads / 2; s > 0; s >>= 1) {
      if (tid < s) {
        VI r = vi_better(VI{sv[tid], si[tid]}, VI{sv[tid + s], si[tid + s]});
        sv[tid] = r.v;
        si[tid] = r.i;
      }
      __syncthreads();
    }
    if (tid == 0) {
      if (!(sv[0] > 0.0)) bad = 1;  // fewer distinct points than control points
      cur = si[0];
    }
    __syncthreads();
    if (bad) break;
  }
  if (tid == 0 && bad) *err = 1;
}

// nearest-other-node distance of every control point
__global__ void k_node_nn(const float4* __restrict__ c0, int N, double* __restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  float4 a = c0[i];
  double best = DBL_MAX;
  for (int k = 0; k < N; k++) {
    if (k == i) continue;
    float4 b = c0[k];
    double d = d2_f64(a.x, a.y, a.z, b.x, b.y, b.z);
    if (d < best) best = d;
  }
  out[i] = sqrt(best);
}

// sum over ordered pairs of the ARAP pair weights exp(-d^2 / (2 (2 sbar)^2)), per row; with a
// sparse graph (adj != nullptr) only over the pairs in it
__global__ void k_arap_rowsum(const float4* __restrict__ c0, int N, double sbar, const uint32_t* __restrict__ adj,
                              int words, double* __restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  float4 a = c0[i];
  double sa = 2.0 * sbar, acc = 0.0;
  for (int k = 0; k < N; k++) {
    if (k == i) continue;
    if (adj && !((adj[(size_t)i * words + (k >> 5)] >> (k & 31)) & 1u)) continue;
    float4 b = c0[k];
    acc += exp(-d2_f64(a.x, a.y, a.z, b.x, b.y, b.z) / (2.0 * sa * sa));
  }
  out[i] = acc;
}

// Sparse ARAP graph: node a keeps its k nearest other nodes (FP64 squared rest distance, ties to
// the lower index), found as k successive minima of (distance, index) above the last one taken;
// both directions of each kept pair are set, so the graph is symmetric. adj starts zeroed.
__global__ void k_node_graph(const float4* __restrict__ c0, int N, int k, uint32_t* __restrict__ adj, int words) {
  int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= N) return;
  const float4 ca = c0[a];
  double last_d = -1.0;
  int last_b = -1;
  for (int r = 0; r < k && r < N - 1; r++) {
    double bd = DBL_MAX;
    int bb = -1;
    for (int b = 0; b < N; b++) {
      if (b == a) continue;
      const float4 cb = c0[b];
      const double d = d2_f64(ca.x, ca.y, ca.z, cb.x, cb.y, cb.z);
      const bool after = d > last_d || (d == last_d && b > last_b);
      if (after && (d < bd || (d == bd && b < bb))) {
        bd = d;
        bb = b;
      }
    }
    if (bb < 0) break;
    atomicOr(&adj[(size_t)a * words + (bb >> 5)], 1u << (bb & 31));
    atomicOr(&adj[(size_t)bb * words + (a >> 5)], 1u << (a & 31));
    last_d = bd;
    last_b = bb;
  }
}

// deterministic single-workgroup sum of n doubles
__global__ __launch_bounds__(1024) void k_sum(const double* __restrict__ v, int n, double* __restrict__ out) {
  __shared__ double sh[1024];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) acc += v[i];
  double r = block_sum_d<1024>(acc, sh);
  if (threadIdx.x == 0) *out = r;
}

// 4 nearest control points (FP64 squared distance, ties to the lower index) and Gaussian blend
// weights exp(-(d^2 - d0^2) / (2 sbar^2)) normalised to 1 (the shift by the nearest d0^2 is a
// common factor that the normalisation removes). Slots beyond N repeat the nearest node with 0.
constexpr int kKnnThreads = 256;
__global__ __launch_bounds__(kKnnThreads) void k_knn(const float* __restrict__ x, const float* __restrict__ y,
                                                     const float* __restrict__ z, int count,
                                                     const float4* __restrict__ c0, int N, double sbar,
                                                     int4* __restrict__ knn, float4* __restrict__ alpha) {
  __shared__ float4 cs[kKnnThreads];
  int j = blockIdx.x * kKnnThreads + threadIdx.x;
  float px = 0.f, py = 0.f, pz = 0.f;
  if (j < count) {
    px = x[j];
    py = y[j];
    pz = z[j];
  }
  double bd[4] = {DBL_MAX, DBL_MAX, DBL_MAX, DBL_MAX};
  int bi[4] = {-1, -1, -1, -1};
  for (int base = 0; base < N; base += kKnnThreads) {
    int k = base + threadIdx.x;
    if (k < N) cs[threadIdx.x] = c0[k];
    __syncthreads();
    int lim = min(kKnnThreads, N - base);
    for (int t = 0; t < lim; t++) {
      float4 c = cs[t];
      double d = d2_f64(px, py, pz, c.x, c.y, c.z);
      if (d < bd[3]) {  // strict: an equal distance keeps the lower (earlier) index
        int pos = 3;
        while (pos > 0 && d < bd[pos - 1]) {
          bd[pos] = bd[pos - 1];
          bi[pos] = bi[pos - 1];
          pos--;
        }
        bd[pos] = d;
        bi[pos] = base + t;
      }
    }
    __syncthreads();
  }
  if (j >= count) return;
  int m = N < 4 ? N : 4;
  double a[4] = {0, 0, 0, 0}, s = 0.0;
  for (int t = 0; t < m; t++) {
    a[t] = exp(-(bd[t] - bd[0]) / (2.0 * sbar * sbar));
    s += a[t];
  }
  for (int t = m; t < 4; t++) bi[t] = bi[0];
  knn[j] = make_int4(bi[0], bi[1], bi[2], bi[3]);
  alpha[j] = make_float4((float)(a[0] / s), (float)(a[1] / s), (float)(a[2] / s), (float)(a[3] / s));
}

// ---------------------------------------------------------------------------------------------
// Target normals: n = (P(u+1,v) - P(u-1,v)) x (P(u,v+1) - P(u,v-1)), normalised, facing the
// camera; stored with the depth as (nx, ny, nz, z). Invalid pixels (border, or any of the five
// depths invalid) get all zeros.

__device__ __forceinline__ bool depth_ok(float z) { return isfinite(z) && z > 0.0f; }

__global__ void k_normal_map(const float* __restrict__ depth, int W, int H, float fx, float fy, float cx,
                             float cy, float4* __restrict__ nmap) {
  int pix = blockIdx.x * blockDim.x + threadIdx.x;
  if (pix >= W * H) return;
  int v = pix / W, u = pix - v * W;
  float4 out = make_float4(0.f, 0.f, 0.f, 0.f);
  if (u >= 1 && v >= 1 && u <= W - 2 && v <= H - 2) {
    float zc = depth[pix], zl = depth[pix - 1], zr = depth[pix + 1], zu = depth[pix - W], zd = depth[pix + W];
    if (depth_ok(zc) && depth_ok(zl) && depth_ok(zr) && depth_ok(zu) && depth_ok(zd)) {
      float ifx = 1.0f / fx, ify = 1.0f / fy;
      f3 Pl = mk3(((float)(u - 1) - cx) * ifx * zl, ((float)v - cy) * ify * zl, zl);
      f3 Pr = mk3(((float)(u + 1) - cx) * ifx * zr, ((float)v - cy) * ify * zr, zr);
      f3 Pu = mk3(((float)u - cx) * ifx * zu, ((float)(v - 1) - cy) * ify * zu, zu);
      f3 Pd = mk3(((float)u - cx) * ifx * zd, ((float)(v + 1) - cy) * ify * zd, zd);
      f3 Pc = mk3(((float)u - cx) * ifx * zc, ((float)v - cy) * ify * zc, zc);
      f3 n = cross(Pr - Pl, Pd - Pu);
      float l = len(n);
      if (l > 0.0f) {
        n = (1.0f / l) * n;
        if (dot(n, Pc) > 0.0f) n = (-1.0f) * n;
        out = make_float4(n.x, n.y, n.z, zc);
      }
    }
  }
  nmap[pix] = out;
}

// ---------------------------------------------------------------------------------------------
// Hamming matching: one wavefront per template feature. Lanes stride over the frame features,
// XOR + popcount the eight 32-bit words, and keep the smallest (distance, index) key; a
// wavefront min-reduction gives the nearest descriptor with ties to the lower index. Lane 0
// gathers the matched frame point and marks the match usable (finite 3D on both sides,
// distance within max_hamming).

constexpr int kMatchThreads = 256;

__global__ __launch_bounds__(kMatchThreads) void k_hamming(const uint4* __restrict__ d1, int K1,
                                                           const uint4* __restrict__ d2, int K2,
                                                           const float* __restrict__ f2xyz, int max_hamming,
                                                           int* __restrict__ midx, int* __restrict__ mdist,
                                                           float4* __restrict__ o2) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = threadIdx.x % kWave;
  const int a = blockIdx.x * (kMatchThreads / kWave) + wave;
  if (a >= K1) return;
  const uint4 q0 = d1[2 * a], q1 = d1[2 * a + 1];
  uint32_t best = 0xFFFFFFFFu;
  for (int b = lane; b < K2; b += kWave) {
    uint4 r0 = d2[2 * b], r1 = d2[2 * b + 1];
    uint32_t d = __builtin_popcount(q0.x ^ r0.x) + __builtin_popcount(q0.y ^ r0.y) +
                 __builtin_popcount(q0.z ^ r0.z) + __builtin_popcount(q0.w ^ r0.w) +
                 __builtin_popcount(q1.x ^ r1.x) + __builtin_popcount(q1.y ^ r1.y) +
                 __builtin_popcount(q1.z ^ r1.z) + __builtin_popcount(q1.w ^ r1.w);
    uint32_t key = (d << 23) | (uint32_t)b;
    best = key < best ? key : best;
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    uint32_t o = __shfl_xor(best, off, kWave);
    best = o < best ? o : best;
  }
  if (lane == 0) {
    int bi = -1, bd = 256;
    if (best != 0xFFFFFFFFu) {
      bi = (int)(best & 0x7FFFFFu);
      bd = (int)(best >> 23);
    }
    midx[a] = bi;
    mdist[a] = bd;
    float4 o = make_float4(0.f, 0.f, 0.f, 0.f);
    if (bi >= 0 && bd <= max_hamming) {
      float x = f2xyz[3 * bi], y = f2xyz[3 * bi + 1], z = f2xyz[3 * bi + 2];
      if (isfinite(x) && isfinite(y) && isfinite(z)) o = make_float4(x, y, z, 1.0f);
    }
    o2[a] = o;
  }
}

// ---------------------------------------------------------------------------------------------
// 1-point RANSAC + reweighting (Sec. 2.1).
//
// k_ransac_sample: compacts the usable matches in index order, then draws min(R, Ku) distinct
// references by a partial Fisher-Yates shuffle driven by SplitMix64 seeded with
// seed + golden * (frame + 1).

constexpr int kSampleThreads = 1024;
constexpr int kSampleLds = 12288;  // usable matches kept in LDS for the shuffle (else it runs in memory)

__global__ __launch_bounds__(kSampleThreads) void k_ransac_sample(const float4* __restrict__ o2, int K1, int R,
                                                                 unsigned long long seed, long long frame,
                                                                 int* __restrict__ ulist, int* __restrict__ refs) {
  __shared__ int scan[kSampleThreads];
  __shared__ int total;
  __shared__ int lst[kSampleLds];
  const bool in_lds = K1 <= kSampleLds;
  if (threadIdx.x == 0) total = 0;
  __syncthreads();
  for (int base = 0; base < K1; base += kSampleThreads) {
    int k = base + threadIdx.x;
    int f = (k < K1 && o2[k].w > 0.0f) ? 1 : 0;
    scan[threadIdx.x] = f;
    __syncthreads();
    for (int off = 1; off < kSampleThreads; off <<= 1) {  // inclusive Hillis-Steele scan
      int v = ((int)threadIdx.x >= off) ? scan[threadIdx.x - off] : 0;
      __syncthreads();
      scan[threadIdx.x] += v;
      __syncthreads();
    }
    if (f) {
      if (in_lds) lst[total + scan[threadIdx.x] - 1] = k;
      else ulist[total + scan[threadIdx.x] - 1] = k;
    }
    __syncthreads();
    if (threadIdx.x == 0) total += scan[kSampleThreads - 1];
    __syncthreads();
  }
  // partial Fisher-Yates over the compacted list, one thread (the draws are sequential); in LDS when
  // the list fits, so that the swaps are not memory round trips
  if (threadIdx.x == 0) {
    int* L = in_lds ? lst : ulist;
    int Ku = total;
    int nh = R < Ku ? R : Ku;
    unsigned long long st = seed + 0x9E3779B97F4A7C15ULL * (unsigned long long)(frame + 1);
    for (int i = 0; i < nh; i++) {
      unsigned long long r = splitmix64_next(&st);
      int j = i + (int)(r % (unsigned long long)(Ku - i));
      int t = L[i];
      L[i] = L[j];
      L[j] = t;
      refs[i] = L[i];
    }
    for (int i = nh; i < R; i++) refs[i] = -1;
  }
}

// One workgroup per hypothesis: Eq. (2) rectifies both point sets about the reference k0; then
// `iters` alternations of the R-step (Eq. (3): weighted rotation fit, FP64, Horn's method) and
// the w-step (Eq. (4): d_k = |S2(k) - R S1(k)|, w_k = min(H / d_k, 1)). Scores W = sum w_k and
// n_in = #{d_k <= H} after the last w-step.
constexpr int kHypThreads = 256;

__global__ __launch_bounds__(kHypThreads) void k_ransac_hyp(const float* __restrict__ f1x, const float* __restrict__ f1y,
                                                            const float* __restrict__ f1z,
                                                            const float4* __restrict__ o2, int K1,
                                                            const int* __restrict__ refs, int iters, double H,
                                                            double* __restrict__ hyp_w, double* __restrict__ hyp_W,
                                                            int* __restrict__ hyp_nin, int* __restrict__ hyp_state) {
  __shared__ double red[9][kHypThreads];
  __shared__ double Rs[9];
  __shared__ int degenerate;
  __shared__ int nin_w[kHypThreads / kWave];
  const int h = blockIdx.x;
  const int k0 = refs[h];
  const int tid = threadIdx.x;
  if (k0 < 0) {
    if (tid == 0) {
      hyp_W[h] = 0.0;
      hyp_nin[h] = 0;
      hyp_state[h] = -1;
    }
    return;
  }
  double* w = hyp_w + (size_t)h * K1;
  const double a0x = f1x[k0], a0y = f1y[k0], a0z = f1z[k0];
  const float4 b0 = o2[k0];
  for (int k = tid; k < K1; k += kHypThreads) w[k] = (o2[k].w > 0.0f) ? 1.0 : 0.0;
  if (tid == 0) degenerate = 0;
  __syncthreads();
  int cnt = 0;  // this thread's matches with d_k <= H in the last w-step
  double Vw[16];  // thread 0: the previous fit's eigenvector basis (the fits warm-start from it)
  for (int it = 0; it < iters; it++) {
    double c[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = tid; k < K1; k += kHypThreads) {
      double wk = w[k];
      if (wk == 0.0) continue;
      float4 b = o2[k];
      double s1[3] = {(double)f1x[k] - a0x, (double)f1y[k] - a0y, (double)f1z[k] - a0z};
      double s2[3] = {(double)b.x - (double)b0.x, (double)b.y - (double)b0.y, (double)b.z - (double)b0.z};
#pragma unroll
      for (int r = 0; r < 3; r++)
#pragma unroll
        for (int q = 0; q < 3; q++) c[r * 3 + q] += wk * s2[r] * s1[q];
    }
#pragma unroll
    for (int e = 0; e < 9; e++) red[e][tid] = c[e];
    __syncthreads();
    for (int s = kHypThreads / 2; s > 0; s >>= 1) {
      if (tid < s)
#pragma unroll
        for (int e = 0; e < 9; e++) red[e][tid] += red[e][tid + s];
      __syncthreads();
    }
    if (tid == 0) {
      double C[9], R[9];
      for (int e = 0; e < 9; e++) C[e] = red[e][0];
      if (rotation_fit_horn(C, R, Vw, it > 0)) degenerate = 1;
      for (int e = 0; e < 9; e++) Rs[e] = R[e];
    }
    __syncthreads();
    if (degenerate) break;
    for (int k = tid; k < K1; k += kHypThreads) {
      float4 b = o2[k];
      if (b.w <= 0.0f) continue;
      double s1[3] = {(double)f1x[k] - a0x, (double)f1y[k] - a0y, (double)f1z[k] - a0z};
      double s2[3] = {(double)b.x - (double)b0.x, (double)b.y - (double)b0.y, (double)b.z - (double)b0.z};
      double e0 = s2[0] - (Rs[0] * s1[0] + Rs[1] * s1[1] + Rs[2] * s1[2]);
      double e1 = s2[1] - (Rs[3] * s1[0] + Rs[4] * s1[1] + Rs[5] * s1[2]);
      double e2 = s2[2] - (Rs[6] * s1[0] + Rs[7] * s1[1] + Rs[8] * s1[2]);
      double d = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
      w[k] = (d > H) ? H / d : 1.0;
      if (it == iters - 1 && d <= H) cnt++;
    }
    __syncthreads();
  }
  if (degenerate) {
    if (tid == 0) {
      hyp_W[h] = 0.0;
      hyp_nin[h] = 0;
      hyp_state[h] = 2;
    }
    return;
  }
  // W = sum w_k over usable matches; n_in = #{d_k <= H} as counted in the last w-step (H / d_k can
  // round to 1 for d_k just above H, so the weight does not decide it)
  double acc = 0.0;
  for (int k = tid; k < K1; k += kHypThreads) {
    if (o2[k].w <= 0.0f) continue;
    acc += w[k];
  }
  red[0][tid] = acc;
  // integer count per wavefront by ballot-free shuffles, then across waves
  int c = cnt;
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) c += __shfl_xor(c, off, kWave);
  if (tid % kWave == 0) nin_w[tid / kWave] = c;
  __syncthreads();
  for (int s = kHypThreads / 2; s > 0; s >>= 1) {
    if (tid < s) red[0][tid] += red[0][tid + s];
    __syncthreads();
  }
  if (tid == 0) {
    int n = 0;
    for (int q = 0; q < kHypThreads / kWave; q++) n += nin_w[q];
    hyp_W[h] = red[0][0];
    hyp_nin[h] = n;
    hyp_state[h] = 0;  // decided in k_ransac_final
  }
}

// Keep the hypotheses whose W reaches half of the best one (a small sum of weights marks an
// outlier reference); w*_k = max of w_k over kept hypotheses; pre-selected iff w* >= 1/2.
__global__ void k_ransac_final(const float4* __restrict__ o2, int K1, int R, const double* __restrict__ hyp_w,
                               const double* __restrict__ hyp_W, int* __restrict__ hyp_state,
                               double* __restrict__ wstar, uint8_t* __restrict__ presel) {
  double Wmax = 0.0;
  for (int h = 0; h < R; h++) {
    int st = hyp_state[h];
    if (st == 0 || st == 1) Wmax = fmax(Wmax, hyp_W[h]);
  }
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < K1) {
    double ws = 0.0;
    bool usable = o2[k].w > 0.0f;
    for (int h = 0; h < R; h++) {
      int st = hyp_state[h];
      if ((st == 0 || st == 1) && hyp_W[h] >= 0.5 * Wmax) ws = fmax(ws, hyp_w[(size_t)h * K1 + k]);
    }
    if (!usable) ws = 0.0;
    wstar[k] = ws;
    presel[k] = (usable && ws >= 0.5) ? 1 : 0;
  }
  __syncthreads();
  // Block 0 records kept (1) / dropped (0). Other blocks may read hyp_state concurrently; they
  // only test "valid" (0 or 1), which this rewrite does not change, so the result is the same
  // whatever the order between blocks.
  if (blockIdx.x == 0) {
    for (int h = threadIdx.x; h < R; h += blockDim.x) {
      int st = hyp_state[h];
      if (st == 0 || st == 1) hyp_state[h] = (hyp_W[h] >= 0.5 * Wmax) ? 1 : 0;
    }
  }
}

}  // namespace

// ---------------------------------------------------------------------------------------------
// launchers

hipError_t launch_fps(const DevState& d, int M, int N, int* err_flag, hipStream_t st) {
  hipLaunchKernelGGL(k_fps, dim3(1), dim3(kFpsThreads), 0, st, d.px, d.py, d.pz, M, N, d.mind, d.node_idx,
                     d.c0, err_flag);
  return hipGetLastError();
}

hipError_t launch_template_tables(DevState& d, hipStream_t st, double* sbar_out, double* sarap_out) {
  // sbar = mean nearest-node distance; s_arap = sum of ARAP pair weights (ordered pairs)
  const int N = d.N;
  double* tmp = d.mind;  // M >= N doubles of scratch
  double* dsum = d.partial;
  if (N == 1) {
    *sbar_out = 1.0;
    *sarap_out = 0.0;
    return hipSuccess;
  }
  hipLaunchKernelGGL(k_node_nn, dim3((N + 255) / 256), dim3(256), 0, st, d.c0, N, tmp);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(1024), 0, st, tmp, N, dsum);
  double s = 0.0;
  hipError_t e = hipMemcpyAsync(&s, dsum, sizeof(double), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  double sbar = s / N;
  hipLaunchKernelGGL(k_arap_rowsum, dim3((N + 255) / 256), dim3(256), 0, st, d.c0, N, sbar, d.adj, d.adj_words,
                     tmp);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(1024), 0, st, tmp, N, dsum);
  double sa = 0.0;
  e = hipMemcpyAsync(&sa, dsum, sizeof(double), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  *sbar_out = sbar;
  *sarap_out = sa;
  return hipGetLastError();
}

hipError_t launch_node_graph(DevState& d, int k, hipStream_t st) {
  if (d.N > 1)
    hipLaunchKernelGGL(k_node_graph, dim3((d.N + 255) / 256), dim3(256), 0, st, d.c0, d.N, k, d.adj, d.adj_words);
  return hipGetLastError();
}

hipError_t launch_knn(const DevState& d, double sbar, hipStream_t st) {
  hipLaunchKernelGGL(k_knn, dim3((d.M + kKnnThreads - 1) / kKnnThreads), dim3(kKnnThreads), 0, st, d.px, d.py,
                     d.pz, d.M, d.c0, d.N, sbar, d.knn, d.alpha);
  if (d.K1 > 0)
    hipLaunchKernelGGL(k_knn, dim3((d.K1 + kKnnThreads - 1) / kKnnThreads), dim3(kKnnThreads), 0, st, d.fpx,
                       d.fpy, d.fpz, d.K1, d.c0, d.N, sbar, d.fknn, d.falpha);
  return hipGetLastError();
}

hipError_t launch_normal_map(const DevState& d, const Intr& K, hipStream_t st) {
  hipLaunchKernelGGL(k_normal_map, dim3((d.HW + 255) / 256), dim3(256), 0, st, d.depth, K.W, K.H, (float)K.fx,
                     (float)K.fy, (float)K.cx, (float)K.cy, d.nmap);
  return hipGetLastError();
}

hipError_t launch_match(const DevState& d, int K2, int max_hamming, hipStream_t st) {
  if (d.K1 == 0) return hipSuccess;
  const int per = kMatchThreads / kWave;
  hipLaunchKernelGGL(k_hamming, dim3((d.K1 + per - 1) / per), dim3(kMatchThreads), 0, st,
                     reinterpret_cast<const uint4*>(d.desc), d.K1, reinterpret_cast<const uint4*>(d.f2desc), K2,
                     d.f2xyz, max_hamming, d.midx, d.mdist, d.o2);
  return hipGetLastError();
}

hipError_t launch_preselect(const DevState& d, int R, int iters, double H, uint64_t seed, int64_t frame,
                            hipStream_t st) {
  if (d.K1 == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ransac_sample, dim3(1), dim3(kSampleThreads), 0, st, d.o2, d.K1, R,
                     (unsigned long long)seed, (long long)frame, d.ulist, d.refs);
  hipLaunchKernelGGL(k_ransac_hyp, dim3(R), dim3(kHypThreads), 0, st, d.fpx, d.fpy, d.fpz, d.o2, d.K1, d.refs,
                     iters, H, d.hyp_w, d.hyp_W, d.hyp_nin, d.hyp_state);
  hipLaunchKernelGGL(k_ransac_final, dim3((d.K1 + 255) / 256), dim3(256), 0, st, d.o2, d.K1, R, d.hyp_w, d.hyp_W,
                     d.hyp_state, d.wstar, d.presel);
  return hipGetLastError();
}
