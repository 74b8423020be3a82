// tt_lm.hip -- one Levenberg-Marquardt iteration of Eq. (1) on the device (Sec. 2):
//
//   k_node_prep        node positions p_i^t = W_i(p_i^0)
//   k_zfill, k_zbuffer (z-buffered association only) the nearest point per pixel
//   k_data_rows        per template point: dual-quaternion blend, nearest-pixel re-projection
//                      (FP64 index math), point-to-plane residual along the target normal, Tukey
//                      weight and the weighted 1x24 Jacobian row; per template feature: the
//                      feature residual, its weight (pre-selected: w*, else the 1 - d/(5H) ramp,
//                      Sec. 2.1) and the weighted 3x24 rows
//   k_lm_scalars       dynamic ARAP weight (Sec. 2): summed data weights over summed pair weights
//   k_arap_assemble    dense ARAP (Sec. 2.2, Eqs. (5)-(6)) over all control-point pairs: one
//                      workgroup per node row writes the row's off-diagonal 6x6 blocks once and
//                      reduces its diagonal block and gradient in LDS
//   k_rows_arap        from the second iteration on (the ARAP weight then fixed), k_arap_assemble
//                      and k_data_rows as one launch (unless their stage timers are on)
//   k_data_assemble    adds the ICP and feature rows into the node-pair blocks through the
//                      static block-CSR (deterministic, no atomics)
//   k_damp             Marquardt damping A + lambda diag(A) + eps I and the right-hand side
//   (Cholesky + solves: tt_chol.hip), or, for the per-node solve,
//   k_node_solve       one 6x6 FP64 Cholesky per node on its diagonal block (only the diagonal
//                      blocks are assembled then)
//   k_update           candidate warps W' = Delta(delta_i) W_i (node-centred increments)
//   k_cost             FP64 cost of the candidate with correspondences and weights frozen (data
//                      and ARAP passes in one launch)
//   k_accept           accept if the cost drops (lambda / 10), else reject (lambda * 10)
//
// Residual rows (all weights frozen within an iteration):
//   ICP     sqrt(omega_j) n . (v_j - q)
//   feature sqrt(w_ORB w_k) (DQB(o1_k) - o2_k)
//   ARAP    per ordered pair (a, b): sqrt(w) (|b| - |e0|), sqrt(w w_angle) (a_hat - b_hat),
//           sqrt(w w_rotation) (qr_a - qr_b), with w = w_ARAP w_ab, e0 = p_b^0 - p_a^0,
//           a = R_a e0, b = p_b^t - p_a^t (the angle of Eq. (6) in chordal form |a_hat - b_hat|).
// FMA contraction only inside one statement (decided by the source, not by the code around an
// inlined body), so that a body compiles to the same arithmetic in every kernel that runs it: the
// single-system and multi-system launches give bit for bit the same results.
#pragma clang fp contract(on)

#include <float.h>

#include "tt_internal.h"
#include "tt_kdtree.h"
#include "tt_math.h"

namespace {

constexpr int kRowThreads = 256;

struct Parts {
  int pts, feat, arap, cdata, carap;  // offsets into the partial-sum buffer
  int nbp, nbf;                       // blocks over points / features
};

__host__ __device__ inline Parts parts_of(int M, int K1, int N) {
  Parts p;
  p.nbp = (M + kRowThreads - 1) / kRowThreads;
  p.nbf = (K1 + kRowThreads - 1) / kRowThreads;
  p.pts = 0;                      // 2 per point block: sum omega, sum omega r^2
  p.feat = p.pts + 2 * p.nbp;     // 2 per feature block: sum w, sum w_orb w |e|^2
  p.arap = p.feat + 2 * p.nbf;    // 1 per node row
  p.cdata = p.arap + N;           // 1 per point/feature block of the candidate
  p.carap = p.cdata + p.nbp + p.nbf;
  return p;
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

__device__ __forceinline__ void load_dq(const float* W, int i, float* q) {
  const float4* p = reinterpret_cast<const float4*>(W + 8 * i);
  float4 a = p[0], b = p[1];
  q[0] = a.x; q[1] = a.y; q[2] = a.z; q[3] = a.w;
  q[4] = b.x; q[5] = b.y; q[6] = b.z; q[7] = b.w;
}

// h(q, y) = G(q)^T y = -u y_w + w y_v + u x y_v
__device__ __forceinline__ f3 gT(const float* q, const float* y) {
  f3 u = mk3(q[1], q[2], q[3]);
  f3 yv = mk3(y[1], y[2], y[3]);
  return (-y[0]) * u + q[0] * yv + cross(u, yv);
}

// y (1x8) times dW/dxi (8x6) of node (q, p): omega part (G(qr)^T y_r + G(qd)^T y_d
// - p x G(qr)^T y_d) / 2, tau part G(qr)^T y_d / 2.
__device__ __forceinline__ void row_times_Q(const float* y, const float* q, f3 p, float coef, float* out6) {
  f3 hr = gT(q, y);
  f3 hd = gT(q + 4, y + 4);
  f3 hrd = gT(q, y + 4);
  f3 om = hr + hd - cross(p, hrd);
  float k = 0.5f * coef;
  out6[0] = k * om.x; out6[1] = k * om.y; out6[2] = k * om.z;
  out6[3] = k * hrd.x; out6[4] = k * hrd.y; out6[5] = k * hrd.z;
}

// ---------------------------------------------------------------------------------------------

__device__ __forceinline__ void node_prep_body(const float* __restrict__ W, const float4* __restrict__ c0,
                                               float4* __restrict__ pos, float4* __restrict__ ndisp, int i) {
  float q[8];
  load_dq(W, i, q);
  float4 c = c0[i];
  f3 dp = dq_disp(q, mk3(c.x, c.y, c.z));
  pos[i] = make_float4(c.x + dp.x, c.y + dp.y, c.z + dp.z, 0.0f);
  ndisp[i] = make_float4(dp.x, dp.y, dp.z, 0.0f);
}
__global__ void k_node_prep(const float* __restrict__ W, const float4* __restrict__ c0, int N,
                            float4* __restrict__ pos, float4* __restrict__ ndisp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) node_prep_body(W, c0, pos, ndisp, i);
}

struct RowArgs {
  // template points
  const float *px, *py, *pz;
  const int4* knn;
  const float4* alpha;
  int M;
  // template features
  const float *fpx, *fpy, *fpz;
  const int4* fknn;
  const float4* falpha;
  int K1;
  const float4* o2;
  const uint8_t* presel;
  const double* wstar;
  // warps
  const float* W;
  const float4* pos;
  // target
  const float4* nmap;
  int Wd, Hd;
  double fx, fy, cx, cy;
  float tukey_c, w_orb, H;
  // z-buffered association (nullptr: every point takes its nearest pixel)
  unsigned long long* zbuf;
  int* zpix;
  KdArgs kd;  // closest-point association (kd.pts null: off)
  // outputs
  int* corr;
  float *rres, *omega, *jac, *wres;
  float *orbw, *jacF, *wresF;
  double* part;
  Parts P;
};

// Nearest-pixel re-projection in FP64 of v = p + d: u = floor(fx x / z + cx + 1/2). Returns
// the pixel or -1.
__device__ __forceinline__ int project_pixel(f3 p, f3 d, const RowArgs& a) {
#pragma clang fp contract(off)
  double x = (double)p.x + (double)d.x, y = (double)p.y + (double)d.y, z = (double)p.z + (double)d.z;
  if (!(z > 0.0)) return -1;
  double uf = a.fx * x / z + a.cx;
  double vf = a.fy * y / z + a.cy;
  double ur = floor(uf + 0.5), vr = floor(vf + 0.5);
  if (!(ur >= 0.0 && ur < (double)a.Wd && vr >= 0.0 && vr < (double)a.Hd)) return -1;
  return (int)vr * a.Wd + (int)ur;
}

// n . (v - q) for v = p + d and the target point q of pixel pix (depth z): p - q is formed in
// FP64 so that only the small residual is rounded to FP32.
__device__ __forceinline__ float plane_residual(f3 p, f3 d, int pix, float4 nm, const RowArgs& a) {
  int vv = pix / a.Wd, uu = pix - vv * a.Wd;
  double z = (double)nm.w;
  double qx = ((double)uu - a.cx) / a.fx * z;
  double qy = ((double)vv - a.cy) / a.fy * z;
  f3 pq = mk3((float)((double)p.x - qx), (float)((double)p.y - qy), (float)((double)p.z - z));
  return dot(mk3(nm.x, nm.y, nm.z), d + pq);
}

// z-buffer pass of the association: every deformed template point that projects into the
// image claims its pixel with the key (float bits of z << 32 | point index); the smallest key
// wins (z > 0, so the float bits order like the values). The pixel is kept for the row pass.
__global__ void k_zfill(unsigned long long* __restrict__ zbuf, int HW) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < HW) zbuf[p] = ~0ull;
}

__global__ __launch_bounds__(kRowThreads) void k_zbuffer(RowArgs a) {
  int j = blockIdx.x * kRowThreads + threadIdx.x;
  if (j >= a.M) return;
  int4 nb = a.knn[j];
  float4 al = a.alpha[j];
  float q0[8], q1[8], q2[8], q3[8];
  load_dq(a.W, nb.x, q0);
  load_dq(a.W, nb.y, q1);
  load_dq(a.W, nb.z, q2);
  load_dq(a.W, nb.w, q3);
  const float alv[4] = {al.x, al.y, al.z, al.w};
  float b[8], sg[4];
  dq_blend4(q0, q1, q2, q3, alv, b, sg);
  f3 p = mk3(a.px[j], a.py[j], a.pz[j]);
  f3 dp = dq_disp(b, p);
  int pix = project_pixel(p, dp, a);
  a.zpix[j] = pix;
  if (pix >= 0) {
    const float z = (float)((double)p.z + (double)dp.z);
    const unsigned long long key = ((unsigned long long)__float_as_uint(z) << 32) | (unsigned)j;
    atomicMin(&a.zbuf[pix], key);
  }
}

__device__ __forceinline__ void data_rows_body(const RowArgs& a, int it, int bx) {
  __shared__ double sh[kRowThreads];
  const int tid = threadIdx.x;
  double s0 = 0.0, s1 = 0.0;
  if (bx < a.P.nbp) {
    // ---- ICP rows of template points
    int j = bx * kRowThreads + tid;
    if (j < a.M) {
      int4 nb = a.knn[j];
      float4 al = a.alpha[j];
      float q0[8], q1[8], q2[8], q3[8];
      load_dq(a.W, nb.x, q0);
      load_dq(a.W, nb.y, q1);
      load_dq(a.W, nb.z, q2);
      load_dq(a.W, nb.w, q3);
      const float alv[4] = {al.x, al.y, al.z, al.w};
      float b[8], sg[4];
      dq_blend4(q0, q1, q2, q3, alv, b, sg);
      f3 p = mk3(a.px[j], a.py[j], a.pz[j]);
      f3 dp = dq_disp(b, p);
      int pix;
      if (a.zbuf) {
        pix = a.zpix[j];  // the pixel of the z-buffer pass; kept only by the point nearest the camera
        if (pix >= 0 && (unsigned)(a.zbuf[pix] & 0xffffffffull) != (unsigned)j) pix = -1;
      } else if (a.kd.pts) {
        const f3 v = p + dp;  // closest-point comparator: the nearest frame point in 3D
        pix = kd_nearest(a.kd, v.x, v.y, v.z);
      } else {
        pix = project_pixel(p, dp, a);
      }
      float r = 0.0f, om = 0.0f;
      f3 n = mk3(0.f, 0.f, 0.f);
      if (pix >= 0) {
        float4 nm = a.nmap[pix];
        if (nm.x != 0.0f || nm.y != 0.0f || nm.z != 0.0f) {
          n = mk3(nm.x, nm.y, nm.z);
          r = plane_residual(p, dp, pix, nm, a);
          if (fabsf(r) < a.tukey_c) {
            float t = r / a.tukey_c;
            om = (1.0f - t * t) * (1.0f - t * t);
          }
        } else {
          pix = -1;
        }
      }
      a.corr[j] = pix;
      a.rres[j] = r;
      a.omega[j] = om;
      float sw = sqrtf(om);
      a.wres[j] = sw * r;
      float J[24];
#pragma unroll
      for (int c = 0; c < 24; c++) J[c] = 0.0f;
      if (om > 0.0f) {
        float Jb[24];
        dq_apply_jac(b, p, Jb);
        float y[8];
#pragma unroll
        for (int c = 0; c < 8; c++) y[c] = n.x * Jb[c] + n.y * Jb[8 + c] + n.z * Jb[16 + c];
        const int nodes[4] = {nb.x, nb.y, nb.z, nb.w};
        const float* qs[4] = {q0, q1, q2, q3};
#pragma unroll
        for (int s = 0; s < 4; s++) {
          float4 ps = a.pos[nodes[s]];
          row_times_Q(y, qs[s], mk3(ps.x, ps.y, ps.z), sw * sg[s] * alv[s], J + 6 * s);
        }
      }
#pragma unroll
      for (int c = 0; c < 24; c += 4)
        *reinterpret_cast<float4*>(a.jac + (size_t)j * 24 + c) = make_float4(J[c], J[c + 1], J[c + 2], J[c + 3]);
      s0 = (double)om;
      s1 = (double)om * (double)r * (double)r;
    }
    double t0 = block_sum_d<kRowThreads>(s0, sh);
    double t1 = block_sum_d<kRowThreads>(s1, sh);
    if (tid == 0) {
      a.part[a.P.pts + 2 * bx] = t0;
      a.part[a.P.pts + 2 * bx + 1] = t1;
    }
  } else {
    // ---- feature rows of template features
    int fb = bx - a.P.nbp;
    int k = fb * kRowThreads + tid;
    if (k < a.K1) {
      float4 o = a.o2[k];
      float w = 0.0f;
      float e[3] = {0.f, 0.f, 0.f};
      float J[72];
#pragma unroll
      for (int c = 0; c < 72; c++) J[c] = 0.0f;
      if (o.w > 0.0f) {
        int4 nb = a.fknn[k];
        float4 al = a.falpha[k];
        float q0[8], q1[8], q2[8], q3[8];
        load_dq(a.W, nb.x, q0);
        load_dq(a.W, nb.y, q1);
        load_dq(a.W, nb.z, q2);
        load_dq(a.W, nb.w, q3);
        const float alv[4] = {al.x, al.y, al.z, al.w};
        float b[8], sg[4];
        dq_blend4(q0, q1, q2, q3, alv, b, sg);
        f3 p = mk3(a.fpx[k], a.fpy[k], a.fpz[k]);
        f3 d = dq_disp(b, p) + (p - mk3(o.x, o.y, o.z));  // DQB(o1) - o2
        if (a.presel[k]) {
          w = (float)a.wstar[k];
        } else {
          float wk = 1.0f - len(d) / (5.0f * a.H);
          w = fminf(fmaxf(wk, 0.0f), 1.0f);
        }
        e[0] = d.x; e[1] = d.y; e[2] = d.z;
        if (w > 0.0f) {
          float sw = sqrtf(a.w_orb * w);
          float Jb[24];
          dq_apply_jac(b, p, Jb);
          const int nodes[4] = {nb.x, nb.y, nb.z, nb.w};
          const float* qs[4] = {q0, q1, q2, q3};
#pragma unroll
          for (int rr = 0; rr < 3; rr++) {
#pragma unroll
            for (int s = 0; s < 4; s++) {
              float4 ps = a.pos[nodes[s]];
              row_times_Q(Jb + 8 * rr, qs[s], mk3(ps.x, ps.y, ps.z), sw * sg[s] * alv[s], J + rr * 24 + 6 * s);
            }
          }
        }
      }
      float sw = sqrtf(a.w_orb * w);
      a.orbw[k] = w;
#pragma unroll
      for (int c = 0; c < 3; c++) a.wresF[(size_t)c * a.K1 + k] = sw * e[c];
#pragma unroll
      for (int c = 0; c < 72; c += 4)
        *reinterpret_cast<float4*>(a.jacF + (size_t)k * 72 + c) = make_float4(J[c], J[c + 1], J[c + 2], J[c + 3]);
      s0 = (double)w;
      s1 = (double)a.w_orb * (double)w * ((double)e[0] * e[0] + (double)e[1] * e[1] + (double)e[2] * e[2]);
    }
    double t0 = block_sum_d<kRowThreads>(s0, sh);
    double t1 = block_sum_d<kRowThreads>(s1, sh);
    if (tid == 0) {
      a.part[a.P.feat + 2 * fb] = t0;
      a.part[a.P.feat + 2 * fb + 1] = t1;
    }
  }
}
__global__ __launch_bounds__(kRowThreads) void k_data_rows(RowArgs a, int it) { data_rows_body(a, it, (int)blockIdx.x); }

// Dynamic ARAP weight, once per frame (iteration 0): lambda_arap times the summed ICP (Tukey)
// and feature (w_ORB w_k) weights over the summed pair weights.
__device__ __forceinline__ void scalars_body(const double* __restrict__ part, Parts P, double lambda_arap,
                                             double w_orb, double s_arap, LMScalars* sc) {
  __shared__ double sh[256];
  double so = 0.0, sw = 0.0;
  for (int b = threadIdx.x; b < P.nbp; b += 256) so += part[P.pts + 2 * b];
  for (int b = threadIdx.x; b < P.nbf; b += 256) sw += part[P.feat + 2 * b];
  so = block_sum_d<256>(so, sh);
  sw = block_sum_d<256>(sw, sh);
  if (threadIdx.x == 0) {
    sc->sum_omega = so;
    sc->sum_orbw = sw;
    sc->w_arap = (s_arap > 0.0) ? lambda_arap * (so + w_orb * sw) / s_arap : 0.0;
  }
}
__global__ __launch_bounds__(256) void k_lm_scalars(const double* __restrict__ part, Parts P, double lambda_arap,
                                                    double w_orb, double s_arap, LMScalars* sc) {
  scalars_body(part, P, lambda_arap, w_orb, s_arap, sc);
}

// ---------------------------------------------------------------------------------------------
// Dense ARAP pair block. For the unordered pair (i, j) both orderings enter; with
// W2 = w_ARAP w_ij, a_hat = R_i e0 / |.|, ap_hat = R_j (-e0) / |.|, b_hat = b / |b|,
// Pb = (I - b_hat b_hat^T) / |b|, Sa = [a_hat]x, Sb = [ap_hat]x:
//   diag (i,i):  omega-omega  W2 wg (I - a a^T) + W2 wr |q_i|^2 I / 2
//                omega-tau    W2 wg Sa Pb
//                tau-tau      2 W2 (b b^T + wg Pb^2)
//   g_i:         omega        -W2 wg (a_hat x b_hat) + W2 wr G(q_i)^T (q_i - q_j)
//                tau          -2 W2 (|b| - |e0|) b_hat + W2 wg Pb (a_hat - ap_hat)
//   off (i,j):   omega-omega  -W2 wr G(q_i)^T G(q_j) / 2
//                omega-tau    -W2 wg Sa Pb
//                tau-omega    W2 wg Pb Sb
//                tau-tau      -2 W2 (b b^T + wg Pb^2)
//   cost:        2 W2 (|b| - |e0|)^2 + W2 wg (|a_hat - b_hat|^2 + |ap_hat + b_hat|^2)
//                + 2 W2 wr |q_i - q_j|^2
struct PairGeom {
  float W2;
  bool geo;
  f3 ah, aph, bh;
  float lb, rlen;
};

// b = p_j - p_i is formed as e0 + (d_j - d_i) from the rest offset and the node displacements,
// and |b| - |e0| as (2 e0 . D + D . D) / (|b| + |e0|), D = d_j - d_i, so that small stretches
// keep their relative precision.
__device__ __forceinline__ PairGeom pair_geom(float4 ci, float4 cj, float4 di, float4 dj, const float* qi,
                                              const float* qj, float w_arap, float inv8s2) {
  PairGeom g;
  f3 e0 = mk3(cj.x - ci.x, cj.y - ci.y, cj.z - ci.z);
  f3 D = mk3(dj.x - di.x, dj.y - di.y, dj.z - di.z);
  f3 bv = e0 + D;
  float e2 = dot(e0, e0);
  g.W2 = w_arap * expf(-e2 * inv8s2);
  f3 av = q_rotate(qi, e0);
  f3 avp = q_rotate(qj, (-1.0f) * e0);
  float la = len(av), lap = len(avp), lb = len(bv), l0 = sqrtf(e2);
  g.geo = (la > 0.0f && lap > 0.0f && lb > 0.0f);
  g.lb = lb;
  g.rlen = g.geo ? (2.0f * dot(e0, D) + dot(D, D)) / (lb + l0) : 0.0f;
  g.ah = g.geo ? (1.0f / la) * av : mk3(0.f, 0.f, 0.f);
  g.aph = g.geo ? (1.0f / lap) * avp : mk3(0.f, 0.f, 0.f);
  g.bh = g.geo ? (1.0f / lb) * bv : mk3(0.f, 0.f, 0.f);
  return g;
}

__device__ __forceinline__ double pair_cost(const PairGeom& g, const float* qi, const float* qj, float wg, float wr) {
  double c = 0.0;
  if (g.geo) {
    f3 d1 = g.ah - g.bh, d2 = g.aph + g.bh;
    c += 2.0 * (double)g.W2 * (double)g.rlen * (double)g.rlen;
    c += (double)g.W2 * (double)wg * ((double)dot(d1, d1) + (double)dot(d2, d2));
  }
  double dq = 0.0;
#pragma unroll
  for (int t = 0; t < 4; t++) dq += (double)(qi[t] - qj[t]) * (double)(qi[t] - qj[t]);
  c += 2.0 * (double)g.W2 * (double)wr * dq;
  return c;
}

// [s]x M for 3x3 M (row-major)
__device__ __forceinline__ void skew_mul(f3 s, const float* M, float* out) {
#pragma unroll
  for (int c = 0; c < 3; c++) {
    float m0 = M[0 * 3 + c], m1 = M[1 * 3 + c], m2 = M[2 * 3 + c];
    out[0 * 3 + c] = -s.z * m1 + s.y * m2;
    out[1 * 3 + c] = s.z * m0 - s.x * m2;
    out[2 * 3 + c] = -s.y * m0 + s.x * m1;
  }
}

struct ArapArgs {
  const float4* c0;
  const float4* ndisp;
  const float* W;
  int N, n, ld;
  float wg, wr, inv8s2;
  const LMScalars* sc;
  float* A;
  float* g;
  double* part;
  Parts P;
  const uint32_t* adj;  // sparse ARAP graph bit rows, nullptr: every pair
  int adj_words;
};

// pair (i, j) is off the sparse ARAP graph: its weight is 0
__device__ __forceinline__ bool off_graph(const ArapArgs& a, int i, int j) {
  return a.adj && !((a.adj[(size_t)i * a.adj_words + (j >> 5)] >> (j & 31)) & 1u);
}

constexpr int kArapThreads = 256;
constexpr int kArapAcc = 36 + 6;

// kOff: also write the off-diagonal blocks (the coupled solve); the per-node solve reads only the
// diagonal blocks and g. kT: threads of the workgroup (128 or 256, a tuning choice).
template <bool kOff, int kT = kArapThreads>
__device__ __forceinline__ void arap_body(const ArapArgs& a, int i) {
  static_assert(kT == 128 || kT == 256, "two or four wavefronts");
  __shared__ float red[kArapAcc][kT + 1];
  __shared__ float wsum[kT / 64][kArapAcc];
  __shared__ double shd[kT];
  const int tid = threadIdx.x;
  const float w_arap = (float)a.sc->w_arap;
  float qi[8];
  load_dq(a.W, i, qi);
  const float4 ci = a.c0[i], pi = a.ndisp[i];
  float D[36], gi[6];
#pragma unroll
  for (int t = 0; t < 36; t++) D[t] = 0.0f;
#pragma unroll
  for (int t = 0; t < 6; t++) gi[t] = 0.0f;
  double cost = 0.0;
  float Gi[12];
  gmat(qi, Gi);
  const float qi2 = qi[0] * qi[0] + qi[1] * qi[1] + qi[2] * qi[2] + qi[3] * qi[3];
  for (int j = tid; j < a.N; j += kT) {
    if (j == i) continue;
    float qj[8];
    load_dq(a.W, j, qj);
    const float4 cj = a.c0[j], pj = a.ndisp[j];
    PairGeom pg = pair_geom(ci, cj, pi, pj, qi, qj, w_arap, a.inv8s2);
    if (off_graph(a, i, j)) pg.W2 = 0.0f;
    const float W2 = pg.W2, wg = a.wg, wr = a.wr;
    if (j > i) cost += pair_cost(pg, qi, qj, wg, wr);
    float Gj[12];
    gmat(qj, Gj);
    // rotation part
    float dqv[4] = {qi[0] - qj[0], qi[1] - qj[1], qi[2] - qj[2], qi[3] - qj[3]};
#pragma unroll
    for (int c = 0; c < 3; c++) {
      D[c * 6 + c] += 0.5f * W2 * wr * qi2;
      gi[c] += W2 * wr * (Gi[0 * 3 + c] * dqv[0] + Gi[1 * 3 + c] * dqv[1] + Gi[2 * 3 + c] * dqv[2] + Gi[3 * 3 + c] * dqv[3]);
    }
    float B[36];
#pragma unroll
    for (int t = 0; t < 36; t++) B[t] = 0.0f;
#pragma unroll
    for (int r = 0; r < 3; r++)
#pragma unroll
      for (int c = 0; c < 3; c++)
        B[r * 6 + c] = -0.5f * W2 * wr *
                       (Gi[0 * 3 + r] * Gj[0 * 3 + c] + Gi[1 * 3 + r] * Gj[1 * 3 + c] + Gi[2 * 3 + r] * Gj[2 * 3 + c] +
                        Gi[3 * 3 + r] * Gj[3 * 3 + c]);
    if (pg.geo) {
      const f3 ah = pg.ah, aph = pg.aph, bh = pg.bh;
      const float ilb = 1.0f / pg.lb;
      const float bb[3] = {bh.x, bh.y, bh.z}, aa[3] = {ah.x, ah.y, ah.z};
      float Pb[9], Pb2[9];
#pragma unroll
      for (int r = 0; r < 3; r++)
#pragma unroll
        for (int c = 0; c < 3; c++) {
          float P = ((r == c) ? 1.0f : 0.0f) - bb[r] * bb[c];
          Pb[r * 3 + c] = P * ilb;
          Pb2[r * 3 + c] = P * ilb * ilb;
        }
      float SaPb[9], SbPb[9], PbSb[9];
      skew_mul(ah, Pb, SaPb);   // Sa Pb
      skew_mul(aph, Pb, SbPb);  // Sb Pb ; Pb Sb = (Sb^T Pb)^T = -(Sb Pb)^T
#pragma unroll
      for (int r = 0; r < 3; r++)
#pragma unroll
        for (int c = 0; c < 3; c++) PbSb[r * 3 + c] = -SbPb[c * 3 + r];
      // diagonal block
#pragma unroll
      for (int r = 0; r < 3; r++)
#pragma unroll
        for (int c = 0; c < 3; c++) {
          float I = (r == c) ? 1.0f : 0.0f;
          D[r * 6 + c] += W2 * wg * (I - aa[r] * aa[c]);
          float wt = W2 * wg * SaPb[r * 3 + c];
          D[r * 6 + 3 + c] += wt;
          D[(3 + c) * 6 + r] += wt;
          D[(3 + r) * 6 + 3 + c] += 2.0f * W2 * (bb[r] * bb[c] + wg * Pb2[r * 3 + c]);
        }
      // gradient
      f3 axb = cross(ah, bh);
      f3 da = ah - aph;
      gi[0] += -W2 * wg * axb.x;
      gi[1] += -W2 * wg * axb.y;
      gi[2] += -W2 * wg * axb.z;
#pragma unroll
      for (int r = 0; r < 3; r++)
        gi[3 + r] += -2.0f * W2 * pg.rlen * bb[r] +
                     W2 * wg * (Pb[r * 3 + 0] * da.x + Pb[r * 3 + 1] * da.y + Pb[r * 3 + 2] * da.z);
      // off-diagonal block (rows i, columns j)
#pragma unroll
      for (int r = 0; r < 3; r++)
#pragma unroll
        for (int c = 0; c < 3; c++) {
          B[r * 6 + 3 + c] = -W2 * wg * SaPb[r * 3 + c];
          B[(3 + r) * 6 + c] = W2 * wg * PbSb[r * 3 + c];
          B[(3 + r) * 6 + 3 + c] = -2.0f * W2 * (bb[r] * bb[c] + wg * Pb2[r * 3 + c]);
        }
    }
    if (kOff && j < i) {
      float* dst = a.A + (size_t)(6 * i) * a.ld + 6 * j;
#pragma unroll
      for (int r = 0; r < 6; r++) {
        float2* d2 = reinterpret_cast<float2*>(dst + (size_t)r * a.ld);
        d2[0] = make_float2(B[r * 6 + 0], B[r * 6 + 1]);
        d2[1] = make_float2(B[r * 6 + 2], B[r * 6 + 3]);
        d2[2] = make_float2(B[r * 6 + 4], B[r * 6 + 5]);
      }
    }
  }
  // reduce the diagonal block, gradient and cost over the workgroup in a fixed order: within each
  // wavefront, lane t < 42 sums entry t of the wavefront's 64 lanes; then the four wavefront sums
#pragma unroll
  for (int t = 0; t < 36; t++) red[t][tid] = D[t];
#pragma unroll
  for (int t = 0; t < 6; t++) red[36 + t][tid] = gi[t];
  shd[tid] = cost;
  __syncthreads();
  const int lane = tid & 63, wv = tid >> 6;
  if (lane < kArapAcc) {
    float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
#pragma unroll
    for (int l = 0; l < 64; l += 4) {
      s0 += red[lane][64 * wv + l];
      s1 += red[lane][64 * wv + l + 1];
      s2 += red[lane][64 * wv + l + 2];
      s3 += red[lane][64 * wv + l + 3];
    }
    wsum[wv][lane] = (s0 + s1) + (s2 + s3);
  }
  __syncthreads();
  if (tid < kArapAcc) {
    float v;
    if constexpr (kT == 256) v = (wsum[0][tid] + wsum[1][tid]) + (wsum[2][tid] + wsum[3][tid]);
    else v = wsum[0][tid] + wsum[1][tid];
    if (tid < 36) {
      const int r = tid / 6, c = tid % 6;
      a.A[(size_t)(6 * i + r) * a.ld + 6 * i + c] = v;
    } else {
      a.g[6 * i + tid - 36] = v;
    }
  } else if (tid == 64) {
    double c = 0.0;
    for (int l = 0; l < kT; l++) c += shd[l];
    a.part[a.P.arap + i] = c;
  }
}
template <bool kOff, int kT>
__global__ __launch_bounds__(kT) void k_arap_assemble(ArapArgs a) {
  arap_body<kOff, kT>(a, (int)blockIdx.x);
}

// From the second LM iteration of a frame on, the ARAP weight is fixed and the dense ARAP blocks and
// the data rows touch disjoint buffers (A, g and the ARAP cost partials; the correspondences,
// residuals, Jacobian rows and data cost partials), so one launch runs both: the N ARAP workgroups
// first (rows of unequal length), then the short rows workgroups, which fill the CUs beside them
// instead of running before them. Each workgroup computes exactly what it computes in its own launch.
static_assert(kRowThreads == kArapThreads, "one block shape for both bodies");
template <bool kOff>
__global__ __launch_bounds__(kArapThreads) void k_rows_arap(ArapArgs aa, RowArgs ra, int it) {
  if ((int)blockIdx.x < aa.N) arap_body<kOff>(aa, (int)blockIdx.x);
  else data_rows_body(ra, it, (int)blockIdx.x - aa.N);
}

// ---------------------------------------------------------------------------------------------
// Data-term blocks through the static block-CSR. Entry = (row index << 5) | (kind << 4) |
// (slot_a << 2) | slot_b; kind 0 = template point (1 row), 1 = template feature (3 rows).
// One wavefront per node-pair block (a >= b): sums J_a^T J_b (and J_a^T r on diagonal blocks
// with slot_a == slot_b), then adds into A and g.

constexpr int kDataThreads = 64;

__device__ __forceinline__ void data_block_body(const int2* __restrict__ blk_ab, const int* __restrict__ blk_ptr,
                                                const uint32_t* __restrict__ ent, const float* __restrict__ jac,
                                                const float* __restrict__ wres, const float* __restrict__ jacF,
                                                const float* __restrict__ wresF, int K1, float* __restrict__ A,
                                                float* __restrict__ g, int ld, int diag_only, int blk) {
  __shared__ float fin[42];
  __shared__ float red[42][kDataThreads + 1];
  const int2 ab = blk_ab[blk];
  if (diag_only && ab.x != ab.y) return;  // whole workgroup: the per-node solve reads no coupling block
  const int lane = threadIdx.x;
  float S[36], G[6];
#pragma unroll
  for (int t = 0; t < 36; t++) S[t] = 0.0f;
#pragma unroll
  for (int t = 0; t < 6; t++) G[t] = 0.0f;
  const int e0 = blk_ptr[blk], e1 = blk_ptr[blk + 1];
  for (int e = e0 + lane; e < e1; e += kDataThreads) {
    uint32_t en = ent[e];
    int sb = en & 3, sa = (en >> 2) & 3, kind = (en >> 4) & 1;
    int idx = (int)(en >> 5);
    if (kind == 0) {
      float Ja[6], Jb[6];
      const float2* ra = reinterpret_cast<const float2*>(jac + (size_t)idx * 24 + 6 * sa);
      const float2* rb = reinterpret_cast<const float2*>(jac + (size_t)idx * 24 + 6 * sb);
#pragma unroll
      for (int c = 0; c < 3; c++) {
        const float2 u = ra[c], v = rb[c];
        Ja[2 * c] = u.x; Ja[2 * c + 1] = u.y;
        Jb[2 * c] = v.x; Jb[2 * c + 1] = v.y;
      }
#pragma unroll
      for (int r = 0; r < 6; r++)
#pragma unroll
        for (int c = 0; c < 6; c++) S[r * 6 + c] += Ja[r] * Jb[c];
      if (sa == sb) {
        float rr = wres[idx];
#pragma unroll
        for (int r = 0; r < 6; r++) G[r] += Ja[r] * rr;
      }
    } else {
#pragma unroll
      for (int q = 0; q < 3; q++) {
        float Ja[6], Jb[6];
        const float2* ra = reinterpret_cast<const float2*>(jacF + (size_t)idx * 72 + q * 24 + 6 * sa);
        const float2* rb = reinterpret_cast<const float2*>(jacF + (size_t)idx * 72 + q * 24 + 6 * sb);
#pragma unroll
        for (int c = 0; c < 3; c++) {
          const float2 u = ra[c], v = rb[c];
          Ja[2 * c] = u.x; Ja[2 * c + 1] = u.y;
          Jb[2 * c] = v.x; Jb[2 * c + 1] = v.y;
        }
#pragma unroll
        for (int r = 0; r < 6; r++)
#pragma unroll
          for (int c = 0; c < 6; c++) S[r * 6 + c] += Ja[r] * Jb[c];
        if (sa == sb) {
          float rr = wresF[(size_t)q * K1 + idx];
#pragma unroll
          for (int r = 0; r < 6; r++) G[r] += Ja[r] * rr;
        }
      }
    }
  }
  // reduction over the wavefront in a fixed order: lane t < 42 sums entry t of all lanes
#pragma unroll
  for (int t = 0; t < 36; t++) red[t][lane] = S[t];
#pragma unroll
  for (int t = 0; t < 6; t++) red[36 + t][lane] = G[t];
  __syncthreads();
  if (lane < 42) {
    float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
#pragma unroll
    for (int l = 0; l < kDataThreads; l += 4) {
      s0 += red[lane][l];
      s1 += red[lane][l + 1];
      s2 += red[lane][l + 2];
      s3 += red[lane][l + 3];
    }
    fin[lane] = (s0 + s1) + (s2 + s3);
  }
  __syncthreads();
  if (lane < 36) {
    int r = lane / 6, c = lane % 6;
    A[(size_t)(6 * ab.x + r) * ld + 6 * ab.y + c] += fin[lane];
  } else if (lane < 42 && ab.x == ab.y) {
    g[6 * ab.x + lane - 36] += fin[lane];
  }
}
__global__ __launch_bounds__(kDataThreads) void k_data_assemble(const int2* __restrict__ blk_ab,
                                                                const int* __restrict__ blk_ptr,
                                                                const uint32_t* __restrict__ ent,
                                                                const float* __restrict__ jac,
                                                                const float* __restrict__ wres,
                                                                const float* __restrict__ jacF,
                                                                const float* __restrict__ wresF, int K1,
                                                                float* __restrict__ A, float* __restrict__ g, int ld,
                                                                int diag_only) {
  data_block_body(blk_ab, blk_ptr, ent, jac, wres, jacF, wresF, K1, A, g, ld, diag_only, (int)blockIdx.x);
}

// Damping A_kk (1 + lambda) + eps, the symmetric diagonal equilibration d_k = 1/sqrt(that) (the
// factorisation scales every entry by d_i d_j when it first reads it, so it factors D A D) and the
// equilibrated right-hand side -d_k g_k. Also totals the cost of the iterate (FP64, fixed order).
__device__ __forceinline__ void damp_body(float* __restrict__ A, const float* __restrict__ g, int n, int npad, int ld,
                                          float* __restrict__ dscale, const double* __restrict__ part, Parts P,
                                          LMScalars* sc) {
  __shared__ float shm[16];
  __shared__ double shd[16];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // the loads are independent, so the unrolled loops keep several in flight at once
  float m = 0.0f;
#pragma unroll 4
  for (int k = tid; k < n; k += 1024) m = fmaxf(m, A[(size_t)k * ld + k]);
  double e = 0.0;
#pragma unroll 2
  for (int b = tid; b < P.nbp; b += 1024) e += part[P.pts + 2 * b + 1];
  for (int b = tid; b < P.nbf; b += 1024) e += part[P.feat + 2 * b + 1];
#pragma unroll 2
  for (int b = tid; b < P.cdata - P.arap; b += 1024) e += part[P.arap + b];
  // within each wavefront by a butterfly, then the sixteen wavefront values in order (the same
  // order on every run)
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    m = fmaxf(m, __shfl_xor(m, off));
    e += __shfl_xor(e, off);
  }
  if (lane == 0) {
    shm[wv] = m;
    shd[wv] = e;
  }
  __syncthreads();
  float mx = shm[0];
  double es = shd[0];
#pragma unroll
  for (int q = 1; q < 16; q++) {
    mx = fmaxf(mx, shm[q]);
    es += shd[q];
  }
  const float eps = 1e-12f * mx;
  const float lam = (float)sc->lambda;
  for (int k = threadIdx.x; k < npad; k += 1024) {
    float d = 1.0f;
    if (k < n) {
      float* dk = A + (size_t)k * ld + k;
      const float a = *dk * (1.0f + lam) + eps;
      *dk = a;
      d = (a > 0.0f) ? 1.0f / sqrtf(a) : 1.0f;
    }
    dscale[k] = d;
    A[(size_t)npad * ld + k] = (k < n) ? -g[k] * d : 0.0f;
  }
  if (threadIdx.x == 0) {
    sc->e_old = es;
    sc->eps = (double)eps;
    sc->chol_fail = 0;
    sc->solve_epoch = (sc->solve_epoch == 0x7FFFFFFF) ? 1 : sc->solve_epoch + 1;
  }
}
__global__ __launch_bounds__(1024) void k_damp(float* __restrict__ A, const float* __restrict__ g, int n, int npad,
                                               int ld, float* __restrict__ dscale, const double* __restrict__ part,
                                               Parts P, LMScalars* sc) {
  damp_body(A, g, n, npad, ld, dscale, part, P, sc);
}

// Per-node step (Sec. 2, each warp W_i updated on its own): node i solves its 6 x 6 diagonal block
// of the damped, equilibrated matrix D A D against its part of the equilibrated right-hand side, by
// Cholesky in FP64 (the block is read from the FP32 lower triangle). One thread per node. A block
// that is not positive definite raises chol_fail, which rejects the step.
__global__ __launch_bounds__(64) void k_node_solve(const float* __restrict__ A, int ld, int npad,
                                                   const float* __restrict__ dscale, int N, float* __restrict__ x,
                                                   LMScalars* sc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int o = 6 * i;
  double ds[6], L[6][6], y[6];
#pragma unroll
  for (int r = 0; r < 6; r++) ds[r] = (double)dscale[o + r];
  bool ok = true;
#pragma unroll
  for (int r = 0; r < 6; r++) {
#pragma unroll
    for (int c = 0; c <= r; c++) {
      double v = (double)A[(size_t)(o + r) * ld + o + c] * ds[r] * ds[c];
#pragma unroll
      for (int k = 0; k < c; k++) v -= L[r][k] * L[c][k];
      if (c == r) {
        ok = ok && (v > 0.0);
        L[r][r] = sqrt(ok ? v : 1.0);
      } else {
        L[r][c] = v / L[c][c];
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 6; r++) {
    double v = (double)A[(size_t)npad * ld + o + r];
#pragma unroll
    for (int k = 0; k < r; k++) v -= L[r][k] * y[k];
    y[r] = v / L[r][r];
  }
#pragma unroll
  for (int r = 5; r >= 0; r--) {
    double v = y[r];
#pragma unroll
    for (int k = r + 1; k < 6; k++) v -= L[k][r] * y[k];
    y[r] = v / L[r][r];
  }
#pragma unroll
  for (int r = 0; r < 6; r++) x[o + r] = ok ? (float)y[r] : 0.0f;
  if (!ok) sc->chol_fail = 1;
}

// Candidate warps from the solution D y of (A + damping) x = -g (y solves the equilibrated system).
__device__ __forceinline__ void update_body(const float* __restrict__ W, const float4* __restrict__ pos,
                                            const float4* __restrict__ c0, const float* __restrict__ x,
                                            const float* __restrict__ dscale, float* __restrict__ Wc,
                                            float4* __restrict__ posc, float4* __restrict__ ndispc, int i) {
  float q[8], out[8];
  load_dq(W, i, q);
  float4 p = pos[i];
  float xi[6];
#pragma unroll
  for (int c = 0; c < 6; c++) xi[c] = x[6 * i + c] * dscale[6 * i + c];
  dq_increment(q, mk3(p.x, p.y, p.z), xi, out);
  float4* d = reinterpret_cast<float4*>(Wc + 8 * i);
  d[0] = make_float4(out[0], out[1], out[2], out[3]);
  d[1] = make_float4(out[4], out[5], out[6], out[7]);
  float4 c = c0[i];
  f3 dc = dq_disp(out, mk3(c.x, c.y, c.z));
  posc[i] = make_float4(c.x + dc.x, c.y + dc.y, c.z + dc.z, 0.0f);
  ndispc[i] = make_float4(dc.x, dc.y, dc.z, 0.0f);
}
__global__ void k_update(const float* __restrict__ W, const float4* __restrict__ pos, const float4* __restrict__ c0,
                         const float* __restrict__ x, const float* __restrict__ dscale, int N, float* __restrict__ Wc,
                         float4* __restrict__ posc, float4* __restrict__ ndispc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) update_body(W, pos, c0, x, dscale, Wc, posc, ndispc, i);
}

// FP64 cost of the candidate with the correspondences, Tukey weights and feature weights of the
// iterate (points: omega (n . (v' - q))^2; features: w_ORB w |DQB(o1) - o2|^2).
__device__ __forceinline__ void cost_data_body(const RowArgs& a, const float* __restrict__ Wc, int bx) {
  __shared__ double sh[kRowThreads];
  const int tid = threadIdx.x;
  double s = 0.0;
  if (bx < a.P.nbp) {
    int j = bx * kRowThreads + tid;
    if (j < a.M) {
      int pix = a.corr[j];
      float om = a.omega[j];
      if (pix >= 0 && om > 0.0f) {
        int4 nb = a.knn[j];
        float4 al = a.alpha[j];
        float q0[8], q1[8], q2[8], q3[8];
        load_dq(Wc, nb.x, q0);
        load_dq(Wc, nb.y, q1);
        load_dq(Wc, nb.z, q2);
        load_dq(Wc, nb.w, q3);
        const float alv[4] = {al.x, al.y, al.z, al.w};
        float b[8], sg[4];
        dq_blend4(q0, q1, q2, q3, alv, b, sg);
        f3 p = mk3(a.px[j], a.py[j], a.pz[j]);
        float r = plane_residual(p, dq_disp(b, p), pix, a.nmap[pix], a);
        s = (double)om * (double)r * (double)r;
      }
    }
  } else {
    int k = (bx - a.P.nbp) * kRowThreads + tid;
    if (k < a.K1) {
      float w = a.orbw[k];
      float4 o = a.o2[k];
      if (o.w > 0.0f && w > 0.0f) {
        int4 nb = a.fknn[k];
        float4 al = a.falpha[k];
        float q0[8], q1[8], q2[8], q3[8];
        load_dq(Wc, nb.x, q0);
        load_dq(Wc, nb.y, q1);
        load_dq(Wc, nb.z, q2);
        load_dq(Wc, nb.w, q3);
        const float alv[4] = {al.x, al.y, al.z, al.w};
        float b[8], sg[4];
        dq_blend4(q0, q1, q2, q3, alv, b, sg);
        f3 p = mk3(a.fpx[k], a.fpy[k], a.fpz[k]);
        f3 d = dq_disp(b, p) + (p - mk3(o.x, o.y, o.z));
        s = (double)a.w_orb * (double)w * ((double)d.x * d.x + (double)d.y * d.y + (double)d.z * d.z);
      }
    }
  }
  double t = block_sum_d<kRowThreads>(s, sh);
  if (tid == 0) a.part[a.P.cdata + bx] = t;
}

__device__ __forceinline__ void cost_arap_body(const ArapArgs& a, const float* __restrict__ Wc,
                                               const float4* __restrict__ ndispc, int i) {
  __shared__ double sh[kArapThreads];
  const float w_arap = (float)a.sc->w_arap;
  float qi[8];
  load_dq(Wc, i, qi);
  const float4 ci = a.c0[i], pi = ndispc[i];
  double cost = 0.0;
  for (int j = i + 1 + threadIdx.x; j < a.N; j += kArapThreads) {
    float qj[8];
    load_dq(Wc, j, qj);
    PairGeom pg = pair_geom(ci, a.c0[j], pi, ndispc[j], qi, qj, w_arap, a.inv8s2);
    if (off_graph(a, i, j)) pg.W2 = 0.0f;
    cost += pair_cost(pg, qi, qj, a.wg, a.wr);
  }
  double t = block_sum_d<kArapThreads>(cost, sh);
  if (threadIdx.x == 0) a.part[a.P.carap + i] = t;
}

// The candidate's data and ARAP cost passes read the frozen correspondences and weights and the
// candidate warps and write disjoint partial sums: one launch, the N ARAP workgroups first (the
// block shape is the one k_rows_arap shares).
__global__ __launch_bounds__(kArapThreads) void k_cost(ArapArgs aa, RowArgs ra, const float* __restrict__ Wc,
                                                       const float4* __restrict__ ndispc) {
  if ((int)blockIdx.x < aa.N) cost_arap_body(aa, Wc, ndispc, (int)blockIdx.x);
  else cost_data_body(ra, Wc, (int)blockIdx.x - aa.N);
}

// Accept / reject on the device: accept iff the factorisation succeeded and the candidate's
// cost is lower. lambda / 10 (>= 1e-10) on accept, * 10 (<= 1e10) on reject.
__device__ __forceinline__ void accept_body(const double* __restrict__ part, Parts P, int N, LMScalars* sc,
                                            float* __restrict__ W, const float* __restrict__ Wc,
                                            float4* __restrict__ pos, const float4* __restrict__ posc,
                                            float4* __restrict__ ndisp, const float4* __restrict__ ndispc,
                                            double* log_old, double* log_new, double* log_lambda, int* log_acc,
                                            double* log_w_arap, int* log_fail) {
  __shared__ double sh[256];
  __shared__ int acc_s;
  double e = 0.0;
  for (int b = threadIdx.x; b < P.nbp + P.nbf; b += 256) e += part[P.cdata + b];
  for (int b = threadIdx.x; b < N; b += 256) e += part[P.carap + b];
  e = block_sum_d<256>(e, sh);
  if (threadIdx.x == 0) {
    int it = sc->it;
    bool fail = sc->chol_fail != 0;
    double e_new = fail ? NAN : e;
    bool acc = !fail && isfinite(e_new) && e_new < sc->e_old;
    log_old[it] = sc->e_old;
    log_new[it] = e_new;
    log_lambda[it] = sc->lambda;
    log_acc[it] = acc ? 1 : 0;
    log_w_arap[it] = sc->w_arap;
    log_fail[it] = fail ? 1 : 0;
    sc->e_new = e_new;
    sc->accept = acc ? 1 : 0;
    sc->lambda = acc ? fmax(sc->lambda / 10.0, 1e-10) : fmin(sc->lambda * 10.0, 1e10);
    sc->it = it + 1;
    acc_s = acc ? 1 : 0;
  }
  __syncthreads();
  if (acc_s) {
    for (int t = threadIdx.x; t < 8 * N; t += 256) W[t] = Wc[t];
    for (int t = threadIdx.x; t < N; t += 256) {
      pos[t] = posc[t];
      ndisp[t] = ndispc[t];
    }
  }
}
__global__ __launch_bounds__(256) void k_accept(const double* __restrict__ part, Parts P, int N, LMScalars* sc,
                                                float* __restrict__ W, const float* __restrict__ Wc,
                                                float4* __restrict__ pos, const float4* __restrict__ posc,
                                                float4* __restrict__ ndisp, const float4* __restrict__ ndispc,
                                                double* log_old, double* log_new, double* log_lambda,
                                                int* log_acc, double* log_w_arap, int* log_fail) {
  accept_body(part, P, N, sc, W, Wc, pos, posc, ndisp, ndispc, log_old, log_new, log_lambda, log_acc, log_w_arap,
              log_fail);
}

__device__ __forceinline__ void lm_begin_body(LMScalars* sc, double lambda0) {
  sc->lambda = lambda0;
  sc->it = 0;
  sc->chol_fail = 0;
  sc->accept = 0;
}
__global__ void k_lm_begin(LMScalars* sc, double lambda0) { lm_begin_body(sc, lambda0); }

// Final deformed template (Sec. 2: interpolation of neighbouring control points) and warps.
__global__ void k_deform_out(const float* __restrict__ px, const float* __restrict__ py, const float* __restrict__ pz,
                             const int4* __restrict__ knn, const float4* __restrict__ alpha, int M,
                             const float* __restrict__ W, int N, float* __restrict__ out_xyz,
                             float* __restrict__ out_dq) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (out_dq && j < 8 * N) out_dq[j] = W[j];
  if (!out_xyz || j >= M) return;
  int4 nb = knn[j];
  float4 al = alpha[j];
  float q0[8], q1[8], q2[8], q3[8];
  load_dq(W, nb.x, q0);
  load_dq(W, nb.y, q1);
  load_dq(W, nb.z, q2);
  load_dq(W, nb.w, q3);
  const float alv[4] = {al.x, al.y, al.z, al.w};
  float b[8], sg[4];
  dq_blend4(q0, q1, q2, q3, alv, b, sg);
  f3 v = dq_apply(b, mk3(px[j], py[j], pz[j]));
  out_xyz[3 * j] = v.x;
  out_xyz[3 * j + 1] = v.y;
  out_xyz[3 * j + 2] = v.z;
}

RowArgs row_args(DevState& d, const tt_params& P, const Intr& K) {
  RowArgs a;
  a.px = d.px; a.py = d.py; a.pz = d.pz; a.knn = d.knn; a.alpha = d.alpha; a.M = d.M;
  a.fpx = d.fpx; a.fpy = d.fpy; a.fpz = d.fpz; a.fknn = d.fknn; a.falpha = d.falpha; a.K1 = d.K1;
  a.o2 = d.o2; a.presel = d.presel; a.wstar = d.wstar;
  a.W = d.W; a.pos = d.pos; a.nmap = d.nmap; a.Wd = K.W; a.Hd = K.H;
  a.fx = K.fx; a.fy = K.fy; a.cx = K.cx; a.cy = K.cy;
  a.tukey_c = (float)P.tukey_c; a.w_orb = (float)P.w_orb; a.H = (float)P.H;
  a.corr = d.corr; a.rres = d.rres; a.omega = d.omega; a.jac = d.jac; a.wres = d.wres;
  a.orbw = d.orbw; a.jacF = d.jacF; a.wresF = d.wresF;
  a.part = d.partial;
  a.P = parts_of(d.M, d.K1, d.N);
  a.zbuf = d.zbuf;
  a.zpix = d.zpix;
  a.kd = KdArgs{d.kd_pts_b ? d.kd_pts : nullptr, d.kd_split, d.kd_count, d.kd_levels};
  return a;
}

ArapArgs arap_args(DevState& d, const tt_params& P) {
  ArapArgs a;
  a.c0 = d.c0; a.ndisp = d.ndisp; a.W = d.W; a.N = d.N; a.n = d.n; a.ld = d.ld;
  a.wg = (float)P.w_angle; a.wr = (float)P.w_rotation;
  double sa = 2.0 * d.sbar;
  a.inv8s2 = (float)(1.0 / (2.0 * sa * sa));
  a.sc = d.sc; a.A = d.A; a.g = d.g; a.part = d.partial;
  a.P = parts_of(d.M, d.K1, d.N);
  a.adj = d.adj;
  a.adj_words = d.adj_words;
  return a;
}

// ---------------------------------------------------------------------------------------------
// Multi-system launches: one launch of a stage over every coupled system of a batch. Each system
// owns a contiguous range of the grid; a workgroup finds its system in the device table by block
// index and runs the single-system kernel's body with the same block-local index, so every system
// gets exactly the results of its own launch. The table is built once per batch composition and
// never changes while launches that read it can run.

struct LMJob {
  static constexpr int kMultiGrids = 5;
  ArapArgs aa;
  RowArgs ra;
  float* W;
  float4 *pos, *ndisp;
  const float4* c0;
  const float* x;
  float *dscale, *Wc;
  float4 *posc, *ndispc;
  LMScalars* sc;
  double* part;
  Parts P;
  int N, n, npad, ld;
  float *A, *g;
  const int2* blk_ab;
  const int* blk_ptr;
  const uint32_t* ent;
  const float *jac, *wres, *jacF, *wresF;
  int K1;
  double *log_old, *log_new, *log_lambda, *log_w_arap;
  int *log_acc, *log_fail;
  double lambda0, lambda_arap, w_orb, s_arap;
  // first workgroup of the system in the node-shaped (64 threads), row-shaped (ARAP rows then
  // point / feature row blocks), data-block, row-block-only and ARAP-only grids
  int start[kMultiGrids];
};

static_assert(LMJob::kMultiGrids == sizeof(LMMulti{}.blocks) / sizeof(int), "one block count per grid");

// the system whose range of grid `kind` holds block b (ranges ascending; empty ranges skipped)
__device__ __forceinline__ int job_of(const LMJob* __restrict__ J, int nj, int kind, int b) {
  int lo = 0, hi = nj - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (J[mid].start[kind] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(64) void k_update_multi(const LMJob* __restrict__ J, int nj) {
  const LMJob& j = J[job_of(J, nj, 0, (int)blockIdx.x)];
  const int i = ((int)blockIdx.x - j.start[0]) * 64 + (int)threadIdx.x;
  if (i < j.N) update_body(j.W, j.pos, j.c0, j.x, j.dscale, j.Wc, j.posc, j.ndispc, i);
}

__global__ __launch_bounds__(kArapThreads) void k_cost_multi(const LMJob* __restrict__ J, int nj) {
  const LMJob& j = J[job_of(J, nj, 1, (int)blockIdx.x)];
  const int bx = (int)blockIdx.x - j.start[1];
  if (bx < j.N) cost_arap_body(j.aa, j.Wc, j.ndispc, bx);
  else cost_data_body(j.ra, j.Wc, bx - j.N);
}

__global__ __launch_bounds__(256) void k_accept_multi(const LMJob* __restrict__ J) {
  const LMJob& j = J[blockIdx.x];
  accept_body(j.part, j.P, j.N, j.sc, j.W, j.Wc, j.pos, j.posc, j.ndisp, j.ndispc, j.log_old, j.log_new,
              j.log_lambda, j.log_acc, j.log_w_arap, j.log_fail);
}

__global__ __launch_bounds__(kArapThreads) void k_rows_arap_multi(const LMJob* __restrict__ J, int nj, int it) {
  const LMJob& j = J[job_of(J, nj, 1, (int)blockIdx.x)];
  const int bx = (int)blockIdx.x - j.start[1];
  if (bx < j.N) arap_body<true>(j.aa, bx);
  else data_rows_body(j.ra, it, bx - j.N);
}

__global__ __launch_bounds__(kDataThreads) void k_data_multi(const LMJob* __restrict__ J, int nj) {
  const LMJob& j = J[job_of(J, nj, 2, (int)blockIdx.x)];
  data_block_body(j.blk_ab, j.blk_ptr, j.ent, j.jac, j.wres, j.jacF, j.wresF, j.K1, j.A, j.g, j.ld, 0,
                  (int)blockIdx.x - j.start[2]);
}

// LM set-up (k_lm_begin on the first workgroup of each system, k_node_prep)
__global__ __launch_bounds__(64) void k_begin_multi(const LMJob* __restrict__ J, int nj) {
  const LMJob& j = J[job_of(J, nj, 0, (int)blockIdx.x)];
  const int lb = (int)blockIdx.x - j.start[0];
  if (lb == 0 && threadIdx.x == 0) lm_begin_body(j.sc, j.lambda0);
  const int i = lb * 64 + (int)threadIdx.x;
  if (i < j.N) node_prep_body(j.W, j.c0, j.pos, j.ndisp, i);
}

// first iteration: the rows, the ARAP weight from them, then the dense ARAP blocks
__global__ __launch_bounds__(kRowThreads) void k_rows_multi(const LMJob* __restrict__ J, int nj, int it) {
  const LMJob& j = J[job_of(J, nj, 3, (int)blockIdx.x)];
  data_rows_body(j.ra, it, (int)blockIdx.x - j.start[3]);
}

__global__ __launch_bounds__(256) void k_scalars_multi(const LMJob* __restrict__ J) {
  const LMJob& j = J[blockIdx.x];
  scalars_body(j.part, j.P, j.lambda_arap, j.w_orb, j.s_arap, j.sc);
}

__global__ __launch_bounds__(kArapThreads) void k_arap_multi(const LMJob* __restrict__ J, int nj) {
  const LMJob& j = J[job_of(J, nj, 4, (int)blockIdx.x)];
  arap_body<true>(j.aa, (int)blockIdx.x - j.start[4]);
}

__global__ __launch_bounds__(1024) void k_damp_multi(const LMJob* __restrict__ J) {
  const LMJob& j = J[blockIdx.x];
  damp_body(j.A, j.g, j.n, j.npad, j.ld, j.dscale, j.part, j.P, j.sc);
}

}  // namespace

size_t lm_multi_bytes(int S) { return sizeof(LMJob) * (size_t)(S > 0 ? S : 0); }

hipError_t lm_multi_fill(DevState* const* ds, const tt_params* const* P, const Intr* K, int S, void* host,
                         void* dev, LMMulti* out) {
  *out = LMMulti{};
  if (S <= 0 || !host || !dev) return hipErrorInvalidValue;
  LMJob* J = static_cast<LMJob*>(host);
  int b[LMJob::kMultiGrids] = {};
  for (int q = 0; q < S; q++) {
    DevState& d = *ds[q];
    if (d.solver == TT_SOLVE_NODE || d.zbuf) return hipErrorInvalidValue;  // extra launches of their own
    LMJob& j = J[q];
    j = LMJob{};
    j.aa = arap_args(d, *P[q]);
    j.ra = row_args(d, *P[q], K[q]);
    j.W = d.W; j.pos = d.pos; j.ndisp = d.ndisp; j.c0 = d.c0;
    j.x = d.x; j.dscale = d.dscale; j.Wc = d.Wc; j.posc = d.posc; j.ndispc = d.ndispc;
    j.sc = d.sc; j.part = d.partial; j.P = parts_of(d.M, d.K1, d.N);
    j.N = d.N; j.n = d.n; j.npad = d.npad; j.ld = d.ld; j.A = d.A; j.g = d.g;
    j.blk_ab = d.blk_ab; j.blk_ptr = d.blk_ptr; j.ent = d.blk_ent;
    j.jac = d.jac; j.wres = d.wres; j.jacF = d.jacF; j.wresF = d.wresF; j.K1 = d.K1;
    j.log_old = d.log_cost_old; j.log_new = d.log_cost_new; j.log_lambda = d.log_lambda;
    j.log_w_arap = d.log_w_arap; j.log_acc = d.log_accept; j.log_fail = d.log_fail;
    j.lambda0 = P[q]->lm_lambda0; j.lambda_arap = P[q]->lambda_arap; j.w_orb = P[q]->w_orb; j.s_arap = d.s_arap;
    const int cnt[LMJob::kMultiGrids] = {(d.N + 63) / 64, d.N + j.P.nbp + j.P.nbf, d.nblk, j.P.nbp + j.P.nbf, d.N};
    for (int k = 0; k < LMJob::kMultiGrids; k++) {
      j.start[k] = b[k];
      b[k] += cnt[k];
    }
  }
  out->jobs = dev;
  out->nj = S;
  for (int k = 0; k < LMJob::kMultiGrids; k++) out->blocks[k] = b[k];
  return hipSuccess;
}

hipError_t lm_multi_build(DevState* const* ds, const tt_params* const* P, const Intr* K, int S, LMMulti* out) {
  *out = LMMulti{};
  if (S <= 0) return hipErrorInvalidValue;
  std::vector<LMJob> J(S);
  void* dev = nullptr;
  hipError_t e = hipMalloc(&dev, lm_multi_bytes(S));
  if (e != hipSuccess) return e;
  e = lm_multi_fill(ds, P, K, S, J.data(), dev, out);
  if (e == hipSuccess) e = hipMemcpy(dev, J.data(), lm_multi_bytes(S), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(dev);
    *out = LMMulti{};
  }
  return e;
}

void lm_multi_free(LMMulti& m) {
  if (m.jobs) (void)hipFree(m.jobs);
  m = LMMulti{};
}

hipError_t launch_lm_multi_begin(const LMMulti& m, hipStream_t st) {
  if (!m.jobs) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_begin_multi, dim3(m.blocks[0]), dim3(64), 0, st, static_cast<const LMJob*>(m.jobs), m.nj);
  return hipGetLastError();
}

hipError_t launch_lm_multi_assemble(const LMMulti& m, int it, hipStream_t st) {
  if (!m.jobs) return hipErrorInvalidValue;
  const LMJob* J = static_cast<const LMJob*>(m.jobs);
  if (it == 0) {  // the ARAP blocks need the ARAP weight from this iteration's rows
    if (m.blocks[3] > 0) hipLaunchKernelGGL(k_rows_multi, dim3(m.blocks[3]), dim3(kRowThreads), 0, st, J, m.nj, it);
    hipLaunchKernelGGL(k_scalars_multi, dim3(m.nj), dim3(256), 0, st, J);
    hipLaunchKernelGGL(k_arap_multi, dim3(m.blocks[4]), dim3(kArapThreads), 0, st, J, m.nj);
  } else {
    hipLaunchKernelGGL(k_rows_arap_multi, dim3(m.blocks[1]), dim3(kArapThreads), 0, st, J, m.nj, it);
  }
  if (m.blocks[2] > 0) hipLaunchKernelGGL(k_data_multi, dim3(m.blocks[2]), dim3(kDataThreads), 0, st, J, m.nj);
  hipLaunchKernelGGL(k_damp_multi, dim3(m.nj), dim3(1024), 0, st, J);
  return hipGetLastError();
}

hipError_t launch_lm_multi_finish(const LMMulti& m, hipStream_t st) {
  if (!m.jobs) return hipErrorInvalidValue;
  const LMJob* J = static_cast<const LMJob*>(m.jobs);
  hipLaunchKernelGGL(k_update_multi, dim3(m.blocks[0]), dim3(64), 0, st, J, m.nj);
  hipLaunchKernelGGL(k_cost_multi, dim3(m.blocks[1]), dim3(kArapThreads), 0, st, J, m.nj);
  hipLaunchKernelGGL(k_accept_multi, dim3(m.nj), dim3(256), 0, st, J);
  return hipGetLastError();
}

int partial_count(int M, int K1, int N) {
  Parts p = parts_of(M, K1, N);
  return p.carap + N;
}

hipError_t launch_lm_begin(DevState& d, double lambda0, hipStream_t st) {
  hipLaunchKernelGGL(k_lm_begin, dim3(1), dim3(1), 0, st, d.sc, lambda0);
  hipLaunchKernelGGL(k_node_prep, dim3((d.N + 63) / 64), dim3(64), 0, st, d.W, d.c0, d.N, d.pos, d.ndisp);
  return hipGetLastError();
}

// Assembly part of an iteration: rows (+ the ARAP weight at iteration 0), dense ARAP blocks,
// data blocks.
hipError_t launch_lm_rows(DevState& d, const tt_params& P, const Intr& K, int it, hipStream_t st) {
  RowArgs ra = row_args(d, P, K);
  if (d.zbuf) {
    hipLaunchKernelGGL(k_zfill, dim3((d.HW + 255) / 256), dim3(256), 0, st, d.zbuf, d.HW);
    hipLaunchKernelGGL(k_zbuffer, dim3((d.M + kRowThreads - 1) / kRowThreads), dim3(kRowThreads), 0, st, ra);
  }
  hipLaunchKernelGGL(k_data_rows, dim3(ra.P.nbp + ra.P.nbf), dim3(kRowThreads), 0, st, ra, it);
  if (it == 0)
    hipLaunchKernelGGL(k_lm_scalars, dim3(1), dim3(256), 0, st, d.partial, ra.P, P.lambda_arap, P.w_orb, d.s_arap,
                       d.sc);
  return hipGetLastError();
}

hipError_t launch_lm_rows_arap(DevState& d, const tt_params& P, const Intr& K, int it, hipStream_t st) {
  if (it == 0) return hipErrorInvalidValue;  // the ARAP weight comes from iteration 0's rows
  RowArgs ra = row_args(d, P, K);
  ArapArgs aa = arap_args(d, P);
  if (d.zbuf) {
    hipLaunchKernelGGL(k_zfill, dim3((d.HW + 255) / 256), dim3(256), 0, st, d.zbuf, d.HW);
    hipLaunchKernelGGL(k_zbuffer, dim3((d.M + kRowThreads - 1) / kRowThreads), dim3(kRowThreads), 0, st, ra);
  }
  const dim3 grid(d.N + ra.P.nbp + ra.P.nbf);
  if (d.solver == TT_SOLVE_NODE)
    hipLaunchKernelGGL(k_rows_arap<false>, grid, dim3(kArapThreads), 0, st, aa, ra, it);
  else
    hipLaunchKernelGGL(k_rows_arap<true>, grid, dim3(kArapThreads), 0, st, aa, ra, it);
  return hipGetLastError();
}

hipError_t launch_lm_arap(DevState& d, const tt_params& P, hipStream_t st) {
  ArapArgs aa = arap_args(d, P);
  const bool off = d.solver != TT_SOLVE_NODE;
  if (d.arap_threads == 128) {
    if (off) hipLaunchKernelGGL((k_arap_assemble<true, 128>), dim3(d.N), dim3(128), 0, st, aa);
    else hipLaunchKernelGGL((k_arap_assemble<false, 128>), dim3(d.N), dim3(128), 0, st, aa);
  } else {
    if (off) hipLaunchKernelGGL((k_arap_assemble<true, kArapThreads>), dim3(d.N), dim3(kArapThreads), 0, st, aa);
    else hipLaunchKernelGGL((k_arap_assemble<false, kArapThreads>), dim3(d.N), dim3(kArapThreads), 0, st, aa);
  }
  return hipGetLastError();
}

hipError_t launch_lm_data(DevState& d, hipStream_t st) {
  if (d.nblk > 0)
    hipLaunchKernelGGL(k_data_assemble, dim3(d.nblk), dim3(kDataThreads), 0, st, d.blk_ab, d.blk_ptr, d.blk_ent,
                       d.jac, d.wres, d.jacF, d.wresF, d.K1, d.A, d.g, d.ld, (int)(d.solver == TT_SOLVE_NODE));
  return hipGetLastError();
}

hipError_t launch_lm_damp(DevState& d, hipStream_t st) {
  Parts p = parts_of(d.M, d.K1, d.N);
  hipLaunchKernelGGL(k_damp, dim3(1), dim3(1024), 0, st, d.A, d.g, d.n, d.npad, d.ld, d.dscale, d.partial, p,
                     d.sc);
  return hipGetLastError();
}

hipError_t launch_node_solve(DevState& d, hipStream_t st) {
  hipLaunchKernelGGL(k_node_solve, dim3((d.N + 63) / 64), dim3(64), 0, st, d.A, d.ld, d.npad, d.dscale, d.N, d.x,
                     d.sc);
  return hipGetLastError();
}

hipError_t launch_lm_finish(DevState& d, const tt_params& P, const Intr& K, hipStream_t st) {
  hipLaunchKernelGGL(k_update, dim3((d.N + 63) / 64), dim3(64), 0, st, d.W, d.pos, d.c0, d.x, d.dscale, d.N, d.Wc,
                     d.posc, d.ndispc);
  RowArgs ra = row_args(d, P, K);
  ArapArgs aa = arap_args(d, P);
  hipLaunchKernelGGL(k_cost, dim3(d.N + ra.P.nbp + ra.P.nbf), dim3(kArapThreads), 0, st, aa, ra, d.Wc, d.ndispc);
  hipLaunchKernelGGL(k_accept, dim3(1), dim3(256), 0, st, d.partial, ra.P, d.N, d.sc, d.W, d.Wc, d.pos, d.posc,
                     d.ndisp, d.ndispc, d.log_cost_old, d.log_cost_new, d.log_lambda, d.log_accept,
                     d.log_w_arap, d.log_fail);
  return hipGetLastError();
}

hipError_t launch_deform_out(const DevState& d, float* out_xyz, float* out_dq, hipStream_t st) {
  int n = d.M > 8 * d.N ? d.M : 8 * d.N;
  hipLaunchKernelGGL(k_deform_out, dim3((n + 255) / 256), dim3(256), 0, st, d.px, d.py, d.pz, d.knn, d.alpha, d.M,
                     d.W, d.N, out_xyz, out_dq);
  return hipGetLastError();
}
