/*
 * tt_oracle.c -- FP64 single-threaded CPU oracle for the per-frame deformation solve of
 * Zhou & Jagadeesan, "Real-time Surface Deformation Recovery from Stereo Videos".
 *
 * TEST INFRASTRUCTURE ONLY (see tt_oracle.h). Plain C99, double precision, one thread, no
 * blocking or fusion: each function restates one step of the method in the order the paper
 * gives it. Where the paper leaves a choice open, the reading taken is stated at the function.
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -fPIC -shared (no FMA contraction, so that every
 * floating-point decision that selects an index is reproducible bit for bit).
 */
#include "tt_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define GOLDEN64 0x9E3779B97F4A7C15ULL

struct tto_stream {
  tto_params P;
  tto_intrinsics K;
  int has_template;
  int M, N, K1, kk;        /* kk = blend slots per point (= P.knn) */
  double* pts;             /* [M*3] template points p_j^0 */
  int32_t* node_idx;       /* [N] template index of each control point */
  double* c0;              /* [N*3] control points at time 0, p_i^0 */
  double sbar;             /* mean nearest-node spacing */
  double s_arap;           /* sum of ARAP pair weights over ordered pairs */
  int32_t* knn_pts;        /* [M*kk] */
  double* alpha_pts;       /* [M*kk] */
  double* f1;              /* [K1*3] template features o^1 */
  uint8_t* desc1;          /* [K1*32] */
  int32_t* knn_feat;       /* [K1*kk] */
  double* alpha_feat;      /* [K1*kk] */
  uint8_t* adj;            /* [N*N] ARAP graph when P.arap_knn > 0 (1 = pair kept), else NULL */
  double* dq;              /* [N*8] current warps W_i^t */
  int64_t frame;
  /* per-frame state, set by tto_frame_begin */
  int frame_ready;
  double* normals;         /* [H*W*3] */
  uint8_t* nvalid;         /* [H*W] */
  double* qpts;            /* [H*W*3] back-projected target points */
  int32_t* midx;           /* [K1] */
  int32_t* mdist;          /* [K1] */
  double* o2;              /* [K1*3] matched frame feature positions o^2 */
  uint8_t* usable;         /* [K1] */
  double* wstar;           /* [K1] */
  uint8_t* presel;         /* [K1] */
  int32_t* hyp_k0;         /* [max(R,1)] */
  double* hyp_W;
  int32_t* hyp_nin;
  uint8_t* hyp_kept;
};

/* ------------------------------------------------------------------------------------------ */
/* small vector helpers                                                                        */

static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
static double norm3(const double* a) { return sqrt(dot3(a, a)); }
/* squared distance, evaluated as dx*dx + dy*dy + dz*dz left to right */
static double dist2(const double* a, const double* b) {
  double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
  return dx * dx + dy * dy + dz * dz;
}
/* [a]x, row-major 3x3 */
static void skew(const double* a, double* S) {
  S[0] = 0;     S[1] = -a[2]; S[2] = a[1];
  S[3] = a[2];  S[4] = 0;     S[5] = -a[0];
  S[6] = -a[1]; S[7] = a[0];  S[8] = 0;
}
static int all_finite3f(const float* a) { return isfinite(a[0]) && isfinite(a[1]) && isfinite(a[2]); }

/* ------------------------------------------------------------------------------------------ */
/* quaternions (w,x,y,z) and dual quaternions [qr | qd]                                          */

static void qmul(const double* a, const double* b, double* c) {
  double w = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
  double x = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
  double y = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
  double z = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
  c[0] = w; c[1] = x; c[2] = y; c[3] = z;
}

/* Rotation of p by quaternion q (not necessarily unit): q p q^* / |q|^2, written as
 * p + (2/|q|^2) (w u x p + u x (u x p)) so that the identity quaternion returns p exactly. */
static void qrotate(const double* q, const double* p, double* out) {
  double s = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
  const double* u = q + 1;
  double up[3], uup[3];
  cross3(u, p, up);
  cross3(u, up, uup);
  for (int c = 0; c < 3; c++) out[c] = p[c] + (2.0 / s) * (q[0] * up[c] + uup[c]);
}

/* Point transform of an 8-vector b treated as a (possibly unnormalised) dual quaternion:
 * v = R(b_r) p + 2 vec(b_d conj(b_r)) / |b_r|^2. This is the warp of a unit dual quaternion and
 * the normalised blend of Kavan et al. for a blended one (Sec. 2: the template follows the
 * interpolation of neighbouring control points, as in DynamicFusion). */
static void dq_apply(const double* b, const double* p, double* v) {
  double w = b[0], e = b[4];
  const double* u = b + 1;
  const double* f = b + 5;
  double s = w * w + u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  double up[3], uup[3], uf[3];
  cross3(u, p, up);
  cross3(u, up, uup);
  cross3(u, f, uf);
  for (int c = 0; c < 3; c++) {
    double X = w * up[c] + uup[c] + w * f[c] - e * u[c] + uf[c];
    v[c] = p[c] + (2.0 / s) * X;
  }
}

/* dv/db (3x8, row-major) of dq_apply at (b, p). With s = |b_r|^2 and
 * X = w u x p + u x (u x p) + w f - e u + u x f, v = p + 2 X / s. */
static void dq_apply_jac(const double* b, const double* p, double* Jb) {
  double w = b[0], e = b[4];
  const double* u = b + 1;
  const double* f = b + 5;
  double s = w * w + u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  double up[3], uup[3], uf[3], X[3];
  cross3(u, p, up);
  cross3(u, up, uup);
  cross3(u, f, uf);
  for (int c = 0; c < 3; c++) X[c] = w * up[c] + uup[c] + w * f[c] - e * u[c] + uf[c];
  double Sp[9], Sf[9], Su[9];
  skew(p, Sp);
  skew(f, Sf);
  skew(u, Su);
  double udp = dot3(u, p);
  /* dX/dw, dX/du (3x3), dX/de, dX/df (3x3) */
  double dXdw[3], dXdu[9], dXde[3], dXdf[9];
  for (int r = 0; r < 3; r++) {
    dXdw[r] = up[r] + f[r];
    dXde[r] = -u[r];
    for (int c = 0; c < 3; c++) {
      double I = (r == c) ? 1.0 : 0.0;
      dXdu[r * 3 + c] = -w * Sp[r * 3 + c] + udp * I + u[r] * p[c] - 2.0 * p[r] * u[c] - e * I - Sf[r * 3 + c];
      dXdf[r * 3 + c] = w * I + Su[r * 3 + c];
    }
  }
  /* dv = (2/s) (dX - X/s ds), ds/dw = 2w, ds/du = 2u, ds/de = ds/df = 0 */
  for (int r = 0; r < 3; r++) {
    double k = 2.0 / s;
    double xs = X[r] / s;
    Jb[r * 8 + 0] = k * (dXdw[r] - xs * 2.0 * w);
    for (int c = 0; c < 3; c++) Jb[r * 8 + 1 + c] = k * (dXdu[r * 3 + c] - xs * 2.0 * u[c]);
    Jb[r * 8 + 4] = k * dXde[r];
    for (int c = 0; c < 3; c++) Jb[r * 8 + 5 + c] = k * dXdf[r * 3 + c];
  }
}

void tto_dq_transform(const double* dq, const double* p, double* out) { dq_apply(dq, p, out); }

void tto_dq_from_rt(const double* qrot, const double* t, double* dq) {
  double tq[4] = {0.0, t[0], t[1], t[2]}, d[4];
  qmul(tq, qrot, d);
  for (int c = 0; c < 4; c++) {
    dq[c] = qrot[c];
    dq[4 + c] = 0.5 * d[c];
  }
}

/* Blend b = sum_k s_k alpha_k W_{n_k}; s_k = -1 when node k's rotation part has a negative dot
 * product with that of the first (nearest) node, so that antipodal representations of the same
 * rotation do not cancel. */
static void dq_blend(const double* dq, const int32_t* nodes, const double* alpha, int k, double* b,
                     double* sgn) {
  const double* r0 = dq + 8 * nodes[0];
  for (int c = 0; c < 8; c++) b[c] = 0.0;
  for (int i = 0; i < k; i++) {
    const double* q = dq + 8 * nodes[i];
    double d = r0[0] * q[0] + r0[1] * q[1] + r0[2] * q[2] + r0[3] * q[3];
    double sg = (d < 0.0) ? -1.0 : 1.0;
    if (sgn) sgn[i] = sg;
    for (int c = 0; c < 8; c++) b[c] += sg * alpha[i] * q[c];
  }
}

void tto_dqb(const double* dq, const int32_t* nodes, const double* alpha, int k, const double* p,
             double* v) {
  double b[8];
  dq_blend(dq, nodes, alpha, k, b, NULL);
  dq_apply(b, p, v);
}

/* G(q) = [-u^T ; w I - [u]x] (4x3): (0,a) * q = G(q) a for a pure quaternion (0,a). */
static void Gmat(const double* q, double* G) {
  double w = q[0];
  const double* u = q + 1;
  G[0] = -u[0]; G[1] = -u[1]; G[2] = -u[2];
  G[3] = w;     G[4] = u[2];  G[5] = -u[1];
  G[6] = -u[2]; G[7] = w;     G[8] = u[0];
  G[9] = u[1];  G[10] = -u[0]; G[11] = w;
}

/* dW_i/dxi_i (8x6, row-major) at xi = 0 for the node-centred increment about node position p:
 * W' = Delta(xi) W with Delta ~ (1 + (0,omega/2), (0, (p x omega + tau)/2)). */
static void dq_increment_jac(const double* W, const double* p, double* Q) {
  double Gr[12], Gd[12], Sp[9];
  Gmat(W, Gr);
  Gmat(W + 4, Gd);
  skew(p, Sp);
  for (int i = 0; i < 48; i++) Q[i] = 0.0;
  for (int r = 0; r < 4; r++) {
    for (int c = 0; c < 3; c++) {
      /* d qr / d omega = G(qr)/2 */
      Q[r * 6 + c] = 0.5 * Gr[r * 3 + c];
      /* d qd / d omega = G(qd)/2 + G(qr) [p]x / 2 ; d qd / d tau = G(qr)/2 */
      double gs = 0.0;
      for (int m = 0; m < 3; m++) gs += Gr[r * 3 + m] * Sp[m * 3 + c];
      Q[(4 + r) * 6 + c] = 0.5 * Gd[r * 3 + c] + 0.5 * gs;
      Q[(4 + r) * 6 + 3 + c] = 0.5 * Gr[r * 3 + c];
    }
  }
}

/* Exp of a rotation vector as a unit quaternion. */
static void quat_exp(const double* om, double* q) {
  double th = norm3(om);
  double k = (th > 1e-10) ? sin(0.5 * th) / th : 0.5 - th * th / 48.0;
  q[0] = cos(0.5 * th);
  q[1] = k * om[0];
  q[2] = k * om[1];
  q[3] = k * om[2];
}

/* Normalise a dual quaternion to unit length with qr.qd = 0, then make qr.w >= 0 (the sign
 * convention that makes the first four components in f_rotation, Eq. (6), well defined). */
static void dq_normalize(double* d) {
  double n = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + d[3] * d[3]);
  for (int c = 0; c < 8; c++) d[c] /= n;
  double rd = d[0] * d[4] + d[1] * d[5] + d[2] * d[6] + d[3] * d[7];
  for (int c = 0; c < 4; c++) d[4 + c] -= rd * d[c];
  if (d[0] < 0.0)
    for (int c = 0; c < 8; c++) d[c] = -d[c];
}

/* W' = Delta(xi) W for the node-centred increment xi = (omega, tau) about p = W(p^0). */
static void dq_increment(const double* W, const double* p, const double* xi, double* out) {
  double qw[4], Rp[3], t[3], D[8];
  quat_exp(xi, qw);
  qrotate(qw, p, Rp);
  for (int c = 0; c < 3; c++) t[c] = p[c] - Rp[c] + xi[3 + c];
  tto_dq_from_rt(qw, t, D);
  double a[4], b[4];
  qmul(D, W, out);                 /* real part: qw * qr */
  qmul(D, W + 4, a);               /* dual part: qw * qd + Dd * qr */
  qmul(D + 4, W, b);
  for (int c = 0; c < 4; c++) out[4 + c] = a[c] + b[c];
  dq_normalize(out);
}

/* ------------------------------------------------------------------------------------------ */
/* random reference sampler: SplitMix64 (Steele, Lea, Flood 2014)                              */

static uint64_t splitmix_next(uint64_t* state) {
  uint64_t z = (*state += GOLDEN64);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

void tto_splitmix64(uint64_t state, int n, uint64_t* out) {
  for (int i = 0; i < n; i++) out[i] = splitmix_next(&state);
}

/* ------------------------------------------------------------------------------------------ */
/* Params and stream                                                                           */

void tto_default_params(tto_params* p) {
  p->num_control_points = 64;
  p->knn = 4;
  p->w_orb = 10.0;        /* Sec. 2, after Eq. (1) */
  p->w_angle = 20.0;      /* Sec. 2.2, after Eq. (5) */
  p->w_rotation = 100.0;  /* Sec. 2.2, after Eq. (5) */
  p->lambda_arap = 1.0;
  p->tukey_c = 5.0;
  p->H = 3.0;
  p->ransac_refs = 30;    /* Sec. 2.1: 30 random references */
  p->ransac_iters = 10;   /* Sec. 2.1: 10 iterations per reference */
  p->lm_iters = 10;
  p->max_hamming = 256;
  p->lm_lambda0 = 1e-4;
  p->seed = 0;
  p->solver = TTO_SOLVE_DENSE;
  p->arap_knn = 0;
  p->assoc_zbuffer = 0;
  p->assoc_kdtree = 0;
}

static void free_frame(tto_stream* s) {
  free(s->normals); free(s->nvalid); free(s->qpts);
  free(s->midx); free(s->mdist); free(s->o2); free(s->usable); free(s->wstar); free(s->presel);
  s->normals = NULL; s->nvalid = NULL; s->qpts = NULL; s->midx = NULL; s->mdist = NULL;
  s->o2 = NULL; s->usable = NULL; s->wstar = NULL; s->presel = NULL;
  s->frame_ready = 0;
}

static void free_template(tto_stream* s) {
  free(s->pts); free(s->node_idx); free(s->c0); free(s->knn_pts); free(s->alpha_pts);
  free(s->f1); free(s->desc1); free(s->knn_feat); free(s->alpha_feat); free(s->dq); free(s->adj);
  s->pts = NULL; s->node_idx = NULL; s->c0 = NULL; s->knn_pts = NULL; s->alpha_pts = NULL;
  s->f1 = NULL; s->desc1 = NULL; s->knn_feat = NULL; s->alpha_feat = NULL; s->dq = NULL; s->adj = NULL;
  s->has_template = 0;
  free_frame(s);
}

int tto_create_stream(const tto_params* p, const tto_intrinsics* K, tto_stream** out) {
  if (!p || !K || !out) return TTO_EINVAL;
  *out = NULL;
  if (p->num_control_points < 1 || p->knn < 1 || p->knn > 8 || p->ransac_refs < 1 ||
      p->ransac_iters < 1 || p->lm_iters < 0 || !(p->H > 0) || !(p->tukey_c > 0) ||
      !(p->w_orb >= 0) || !(p->w_angle >= 0) || !(p->w_rotation >= 0) || !(p->lambda_arap >= 0) ||
      !(p->lm_lambda0 > 0) || (p->solver != TTO_SOLVE_DENSE && p->solver != TTO_SOLVE_NODE) ||
      p->arap_knn < 0 || p->arap_knn > 32 || (p->assoc_zbuffer != 0 && p->assoc_zbuffer != 1) ||
      (p->assoc_kdtree != 0 && p->assoc_kdtree != 1) || (p->assoc_kdtree && p->assoc_zbuffer))
    return TTO_EINVAL;
  if (K->width < 3 || K->height < 3 || !(K->fx > 0) || !(K->fy > 0) || !isfinite(K->cx) ||
      !isfinite(K->cy))
    return TTO_EINVAL;
  tto_stream* s = (tto_stream*)calloc(1, sizeof(tto_stream));
  if (!s) return TTO_ENOMEM;
  s->P = *p;
  s->K = *K;
  int R = p->ransac_refs > 0 ? p->ransac_refs : 1;
  s->hyp_k0 = (int32_t*)malloc(sizeof(int32_t) * R);
  s->hyp_W = (double*)malloc(sizeof(double) * R);
  s->hyp_nin = (int32_t*)malloc(sizeof(int32_t) * R);
  s->hyp_kept = (uint8_t*)malloc(R);
  if (!s->hyp_k0 || !s->hyp_W || !s->hyp_nin || !s->hyp_kept) {
    tto_destroy(s);
    return TTO_ENOMEM;
  }
  *out = s;
  return TTO_OK;
}

int tto_destroy(tto_stream* s) {
  if (!s) return TTO_EINVAL;
  free_template(s);
  free(s->hyp_k0); free(s->hyp_W); free(s->hyp_nin); free(s->hyp_kept);
  free(s);
  return TTO_OK;
}

/* ------------------------------------------------------------------------------------------ */
/* Template (Sec. 2: sparse control points on the template; each point follows the interpolation
 * of neighbouring control points)                                                              */

/* k nearest nodes of point x by squared distance, ties to the lower node index, with Gaussian
 * blend weights exp(-d^2 / (2 sbar^2)) normalised to sum 1. The exponent is shifted by the
 * nearest node's d^2 (a common factor that the normalisation removes) so that far points do
 * not underflow. Slots beyond N hold the nearest node with weight 0. */
static void knn_blend(const double* c0, int N, double sbar, const double* x, int kk, int32_t* idx,
                      double* alpha) {
  double bestd[8];
  int m = kk < N ? kk : N;
  for (int t = 0; t < m; t++) { idx[t] = -1; bestd[t] = INFINITY; }
  for (int i = 0; i < N; i++) {
    double d = dist2(x, c0 + 3 * i);
    /* insert into sorted list; strict < keeps the lower index first among equals */
    int pos = m;
    while (pos > 0 && (idx[pos - 1] < 0 || d < bestd[pos - 1])) pos--;
    if (pos < m) {
      for (int t = m - 1; t > pos; t--) { bestd[t] = bestd[t - 1]; idx[t] = idx[t - 1]; }
      bestd[pos] = d;
      idx[pos] = i;
    }
  }
  double sum = 0.0;
  for (int t = 0; t < m; t++) {
    alpha[t] = exp(-(bestd[t] - bestd[0]) / (2.0 * sbar * sbar));
    sum += alpha[t];
  }
  for (int t = 0; t < m; t++) alpha[t] /= sum;
  for (int t = m; t < kk; t++) { idx[t] = idx[0]; alpha[t] = 0.0; }
}

static double arap_pair_weight(const tto_stream* s, int a, int b) {
  /* w_{i1,i2}: larger for control points that are closer at time 0 (Sec. 2.2); Gaussian of
   * the rest distance with sigma = 2 sbar. With a sparse ARAP graph, 0 off the graph. */
  if (s->adj && !s->adj[(size_t)a * s->N + b]) return 0.0;
  double sa = 2.0 * s->sbar;
  return exp(-dist2(s->c0 + 3 * a, s->c0 + 3 * b) / (2.0 * sa * sa));
}

int tto_set_template(tto_stream* s, const float* pts_xyz, int M, const float* feat_xyz,
                     const uint8_t* feat_desc, int K1) {
  if (!s || !pts_xyz || M < 1 || K1 < 0 || (K1 > 0 && (!feat_xyz || !feat_desc))) return TTO_EINVAL;
  int N = s->P.num_control_points;
  if (N > M) return TTO_EINVAL;
  for (int j = 0; j < M; j++)
    if (!all_finite3f(pts_xyz + 3 * j)) return TTO_EINVAL;
  for (int k = 0; k < K1; k++)
    if (!all_finite3f(feat_xyz + 3 * k)) return TTO_EINVAL;
  free_template(s);
  int kk = s->P.knn;
  s->M = M; s->N = N; s->K1 = K1; s->kk = kk;
  s->pts = (double*)malloc(sizeof(double) * 3 * M);
  s->node_idx = (int32_t*)malloc(sizeof(int32_t) * N);
  s->c0 = (double*)malloc(sizeof(double) * 3 * N);
  s->knn_pts = (int32_t*)malloc(sizeof(int32_t) * M * kk);
  s->alpha_pts = (double*)malloc(sizeof(double) * M * kk);
  s->f1 = (double*)malloc(sizeof(double) * 3 * (K1 ? K1 : 1));
  s->desc1 = (uint8_t*)malloc(32 * (K1 ? K1 : 1));
  s->knn_feat = (int32_t*)malloc(sizeof(int32_t) * (K1 ? K1 : 1) * kk);
  s->alpha_feat = (double*)malloc(sizeof(double) * (K1 ? K1 : 1) * kk);
  s->dq = (double*)malloc(sizeof(double) * 8 * N);
  double* mind = (double*)malloc(sizeof(double) * M);
  if (!s->pts || !s->node_idx || !s->c0 || !s->knn_pts || !s->alpha_pts || !s->f1 || !s->desc1 ||
      !s->knn_feat || !s->alpha_feat || !s->dq || !mind) {
    free(mind);
    free_template(s);
    return TTO_ENOMEM;
  }
  for (int j = 0; j < 3 * M; j++) s->pts[j] = (double)pts_xyz[j];
  for (int k = 0; k < 3 * K1; k++) s->f1[k] = (double)feat_xyz[k];
  if (K1) memcpy(s->desc1, feat_desc, 32 * (size_t)K1);

  /* Control points by farthest-point sampling: start at point 0; each next point maximises
   * the squared distance to the nearest chosen one, ties to the lower index. */
  for (int j = 0; j < M; j++) mind[j] = INFINITY;
  int cur = 0;
  for (int i = 0; i < N; i++) {
    s->node_idx[i] = cur;
    for (int c = 0; c < 3; c++) s->c0[3 * i + c] = s->pts[3 * cur + c];
    if (i == N - 1) break;
    double best = -1.0;
    int bi = -1;
    for (int j = 0; j < M; j++) {
      double d = dist2(s->pts + 3 * j, s->c0 + 3 * i);
      if (d < mind[j]) mind[j] = d;
      if (mind[j] > best) { best = mind[j]; bi = j; }
    }
    if (!(best > 0.0)) { /* fewer distinct points than control points */
      free(mind);
      free_template(s);
      return TTO_EINVAL;
    }
    cur = bi;
  }
  free(mind);

  /* mean spacing: average over nodes of the distance to the nearest other node */
  if (N == 1) {
    s->sbar = 1.0;
  } else {
    double acc = 0.0;
    for (int i = 0; i < N; i++) {
      double best = INFINITY;
      for (int k = 0; k < N; k++) {
        if (k == i) continue;
        double d = dist2(s->c0 + 3 * i, s->c0 + 3 * k);
        if (d < best) best = d;
      }
      acc += sqrt(best);
    }
    s->sbar = acc / N;
  }
  for (int j = 0; j < M; j++)
    knn_blend(s->c0, N, s->sbar, s->pts + 3 * j, kk, s->knn_pts + kk * j, s->alpha_pts + kk * j);
  for (int k = 0; k < K1; k++)
    knn_blend(s->c0, N, s->sbar, s->f1 + 3 * k, kk, s->knn_feat + kk * k, s->alpha_feat + kk * k);
  /* Sparse ARAP graph (the alternative to the dense connection of Sec. 2.2): node a keeps its
   * arap_knn nearest other nodes (squared rest distance, ties to the lower index), and a pair is
   * kept if either node keeps the other. */
  if (s->P.arap_knn > 0) {
    s->adj = (uint8_t*)calloc((size_t)N * N, 1);
    if (!s->adj) {
      free_template(s);
      return TTO_ENOMEM;
    }
    for (int a = 0; a < N; a++) {
      for (int r = 0; r < s->P.arap_knn && r < N - 1; r++) {
        int best = -1;
        double bd = INFINITY;
        for (int b = 0; b < N; b++) {
          if (b == a || s->adj[(size_t)a * N + b] == 2) continue;
          double d = dist2(s->c0 + 3 * a, s->c0 + 3 * b);
          if (d < bd) { bd = d; best = b; }
        }
        s->adj[(size_t)a * N + best] = 2; /* chosen by a */
      }
    }
    for (int a = 0; a < N; a++)
      for (int b = 0; b < N; b++)
        if (s->adj[(size_t)a * N + b] == 2 || s->adj[(size_t)b * N + a] == 2) {
          s->adj[(size_t)a * N + b] |= 1;
          s->adj[(size_t)b * N + a] |= 1;
        }
  }
  /* sum of ARAP weights over all ordered pairs (used to scale the dynamic ARAP weight) */
  double sa = 0.0;
  for (int a = 0; a < N; a++)
    for (int b = 0; b < N; b++)
      if (a != b) sa += arap_pair_weight(s, a, b);
  s->s_arap = sa;
  for (int i = 0; i < N; i++) {
    double* d = s->dq + 8 * i;
    for (int c = 0; c < 8; c++) d[c] = 0.0;
    d[0] = 1.0;
  }
  s->frame = 0;
  s->has_template = 1;
  return TTO_OK;
}

int tto_num_nodes(const tto_stream* s) { return (s && s->has_template) ? s->N : 0; }

int tto_get_template_info(const tto_stream* s, int32_t* node_idx, int32_t* knn_pts,
                          double* alpha_pts, int32_t* knn_feat, double* alpha_feat,
                          double* sbar, double* s_arap) {
  if (!s) return TTO_EINVAL;
  if (!s->has_template) return TTO_ESTATE;
  if (node_idx) memcpy(node_idx, s->node_idx, sizeof(int32_t) * s->N);
  if (knn_pts) memcpy(knn_pts, s->knn_pts, sizeof(int32_t) * s->M * s->kk);
  if (alpha_pts) memcpy(alpha_pts, s->alpha_pts, sizeof(double) * s->M * s->kk);
  if (knn_feat && s->K1) memcpy(knn_feat, s->knn_feat, sizeof(int32_t) * s->K1 * s->kk);
  if (alpha_feat && s->K1) memcpy(alpha_feat, s->alpha_feat, sizeof(double) * s->K1 * s->kk);
  if (sbar) *sbar = s->sbar;
  if (s_arap) *s_arap = s->s_arap;
  return TTO_OK;
}

int tto_get_state(const tto_stream* s, double* dq, int64_t* frame) {
  if (!s) return TTO_EINVAL;
  if (!s->has_template) return TTO_ESTATE;
  if (dq) memcpy(dq, s->dq, sizeof(double) * 8 * s->N);
  if (frame) *frame = s->frame;
  return TTO_OK;
}

int tto_set_state(tto_stream* s, const double* dq, int64_t frame) {
  if (!s || frame < 0) return TTO_EINVAL;
  if (!s->has_template) return TTO_ESTATE;
  if (dq) {
    for (int i = 0; i < 8 * s->N; i++)
      if (!isfinite(dq[i])) return TTO_EINVAL;
    memcpy(s->dq, dq, sizeof(double) * 8 * s->N);
  }
  s->frame = frame;
  return TTO_OK;
}

/* ------------------------------------------------------------------------------------------ */
/* Target normals (Sec. 2: only the distance along the normal direction enters f_ICP)          */

static int depth_ok(float z) { return isfinite(z) && z > 0.0f; }

static void backproject(const tto_intrinsics* K, int u, int v, double z, double* P) {
  P[0] = ((double)u - K->cx) / K->fx * z;
  P[1] = ((double)v - K->cy) / K->fy * z;
  P[2] = z;
}

/* Normal by central differences of back-projected neighbours, n = (P(u+1,v) - P(u-1,v)) x
 * (P(u,v+1) - P(u,v-1)), normalised and oriented towards the camera (n . P < 0). A pixel has a
 * normal if it and its four neighbours have valid depth and it is not on the border. */
void tto_normal_map(const float* depth, const tto_intrinsics* K, double* normals, uint8_t* valid) {
  int W = K->width, H = K->height;
  for (int v = 0; v < H; v++) {
    for (int u = 0; u < W; u++) {
      int pix = v * W + u;
      double* n = normals + 3 * pix;
      n[0] = n[1] = n[2] = 0.0;
      valid[pix] = 0;
      if (u < 1 || v < 1 || u > W - 2 || v > H - 2) continue;
      if (!depth_ok(depth[pix]) || !depth_ok(depth[pix - 1]) || !depth_ok(depth[pix + 1]) ||
          !depth_ok(depth[pix - W]) || !depth_ok(depth[pix + W]))
        continue;
      double Pl[3], Pr[3], Pu[3], Pd[3], Pc[3], du[3], dv[3], c[3];
      backproject(K, u - 1, v, depth[pix - 1], Pl);
      backproject(K, u + 1, v, depth[pix + 1], Pr);
      backproject(K, u, v - 1, depth[pix - W], Pu);
      backproject(K, u, v + 1, depth[pix + W], Pd);
      backproject(K, u, v, depth[pix], Pc);
      for (int k = 0; k < 3; k++) { du[k] = Pr[k] - Pl[k]; dv[k] = Pd[k] - Pu[k]; }
      cross3(du, dv, c);
      double l = norm3(c);
      if (!(l > 0.0)) continue;
      for (int k = 0; k < 3; k++) c[k] /= l;
      if (dot3(c, Pc) > 0.0)
        for (int k = 0; k < 3; k++) c[k] = -c[k];
      n[0] = c[0]; n[1] = c[1]; n[2] = c[2];
      valid[pix] = 1;
    }
  }
}

/* ------------------------------------------------------------------------------------------ */
/* ORB matching (Sec. 2.1): template features matched to the live frame                       */

static int popcount8(uint8_t x) {
  int c = 0;
  while (x) { c += x & 1u; x >>= 1; }
  return c;
}

void tto_hamming_match(const uint8_t* desc1, int K1, const uint8_t* desc2, int K2, int32_t* idx,
                       int32_t* dist) {
  for (int a = 0; a < K1; a++) {
    int best = 257, bi = -1;
    for (int b = 0; b < K2; b++) {
      int d = 0;
      for (int t = 0; t < 32; t++) d += popcount8((uint8_t)(desc1[32 * a + t] ^ desc2[32 * b + t]));
      if (d < best) { best = d; bi = b; }
    }
    idx[a] = bi;
    dist[a] = (bi < 0) ? 256 : best;
  }
}

/* ------------------------------------------------------------------------------------------ */
/* Rotation fit for Eq. (3): argmax tr(R^T M) over SO(3), M = sum_k w_k S2(k) S1(k)^T          */

/* Cyclic Jacobi eigen-decomposition of a symmetric 3x3 matrix: A = V diag(e) V^T. */
static void jacobi3(const double* Ain, double* e, double* V) {
  double A[9];
  memcpy(A, Ain, sizeof(A));
  for (int i = 0; i < 9; i++) V[i] = (i % 4 == 0) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 64; sweep++) {
    double off = A[1] * A[1] + A[2] * A[2] + A[5] * A[5];
    double diag = A[0] * A[0] + A[4] * A[4] + A[8] * A[8];
    if (off <= 1e-40 * diag || off == 0.0) break;
    for (int p = 0; p < 2; p++) {
      for (int q = p + 1; q < 3; q++) {
        double apq = A[3 * p + q];
        if (apq == 0.0) continue;
        double app = A[3 * p + p], aqq = A[3 * q + q];
        double theta = (aqq - app) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
        /* A <- G^T A G with G the rotation in the (p,q) plane */
        for (int k = 0; k < 3; k++) {
          double akp = A[3 * k + p], akq = A[3 * k + q];
          A[3 * k + p] = c * akp - sn * akq;
          A[3 * k + q] = sn * akp + c * akq;
        }
        for (int k = 0; k < 3; k++) {
          double apk = A[3 * p + k], aqk = A[3 * q + k];
          A[3 * p + k] = c * apk - sn * aqk;
          A[3 * q + k] = sn * apk + c * aqk;
        }
        for (int k = 0; k < 3; k++) {
          double vkp = V[3 * k + p], vkq = V[3 * k + q];
          V[3 * k + p] = c * vkp - sn * vkq;
          V[3 * k + q] = sn * vkp + c * vkq;
        }
      }
    }
  }
  e[0] = A[0]; e[1] = A[4]; e[2] = A[8];
}

static double det3(const double* A) {
  return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
         A[2] * (A[3] * A[7] - A[4] * A[6]);
}

/* SVD M = U diag(sigma) V^T from the eigen-decomposition of M^T M; the optimal rotation is
 * U diag(1, 1, det(U V^T)) V^T (Kabsch / Umeyama). Degenerate (returns 1) when
 * sigma_2 < 1e-9 sigma_1, i.e. the matches do not fix a rotation. */
int tto_rotation_fit(const double* M, double* R, double* sigma) {
  double MtM[9], e[3], V[9];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      double a = 0.0;
      for (int k = 0; k < 3; k++) a += M[3 * k + i] * M[3 * k + j];
      MtM[3 * i + j] = a;
    }
  jacobi3(MtM, e, V);
  /* sort eigenpairs descending */
  int ord[3] = {0, 1, 2};
  for (int i = 0; i < 3; i++)
    for (int j = i + 1; j < 3; j++)
      if (e[ord[j]] > e[ord[i]]) { int t = ord[i]; ord[i] = ord[j]; ord[j] = t; }
  double Vs[9], sg[3];
  for (int c = 0; c < 3; c++) {
    sg[c] = sqrt(e[ord[c]] > 0.0 ? e[ord[c]] : 0.0);
    for (int r = 0; r < 3; r++) Vs[3 * r + c] = V[3 * r + ord[c]];
  }
  if (sigma) { sigma[0] = sg[0]; sigma[1] = sg[1]; sigma[2] = sg[2]; }
  for (int i = 0; i < 9; i++) R[i] = (i % 4 == 0) ? 1.0 : 0.0;
  if (!(sg[0] > 0.0) || sg[1] < 1e-9 * sg[0]) return 1;
  /* U_c = M V_c / sigma_c for the two leading columns; U_3 completes a right-handed frame */
  double U[9];
  for (int c = 0; c < 2; c++)
    for (int r = 0; r < 3; r++) {
      double a = 0.0;
      for (int k = 0; k < 3; k++) a += M[3 * r + k] * Vs[3 * k + c];
      U[3 * r + c] = a / sg[c];
    }
  double u1[3] = {U[0], U[3], U[6]}, u2[3] = {U[1], U[4], U[7]}, u3[3];
  cross3(u1, u2, u3);
  U[2] = u3[0]; U[5] = u3[1]; U[8] = u3[2];
  double d = (det3(U) * det3(Vs) < 0.0) ? -1.0 : 1.0;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++)
      R[3 * i + j] = U[3 * i + 0] * Vs[3 * j + 0] + U[3 * i + 1] * Vs[3 * j + 1] + d * U[3 * i + 2] * Vs[3 * j + 2];
  return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* 1-point RANSAC + reweighting pre-selection (Sec. 2.1, Eqs. (2)-(4))                          */

int tto_preselect(const double* o1, const double* o2, const uint8_t* usable, int K, double H,
                  int refs, int iters, uint64_t seed, int64_t frame, double* wstar,
                  uint8_t* preselected, int32_t* hyp_k0, double* hyp_W, int32_t* hyp_nin,
                  uint8_t* hyp_kept) {
  int* U = (int*)malloc(sizeof(int) * (K ? K : 1));
  double* w = (double*)malloc(sizeof(double) * (K ? K : 1));
  double* d = (double*)malloc(sizeof(double) * (K ? K : 1));
  double* S1 = (double*)malloc(sizeof(double) * 3 * (K ? K : 1));
  double* S2 = (double*)malloc(sizeof(double) * 3 * (K ? K : 1));
  int Ku = 0;
  for (int k = 0; k < K; k++)
    if (usable[k]) U[Ku++] = k;
  for (int k = 0; k < K; k++) { wstar[k] = 0.0; preselected[k] = 0; }
  /* the references: every usable match (exhaustive) or min(refs, Ku) distinct random matches
   * drawn by a partial Fisher-Yates shuffle driven by SplitMix64 */
  int nh;
  if (refs == 0) {
    nh = Ku;
  } else {
    nh = refs < Ku ? refs : Ku;
    uint64_t st = seed + GOLDEN64 * (uint64_t)(frame + 1);
    for (int i = 0; i < nh; i++) {
      uint64_t r = splitmix_next(&st);
      int j = i + (int)(r % (uint64_t)(Ku - i));
      int t = U[i]; U[i] = U[j]; U[j] = t;
    }
  }
  int hyp_total = refs == 0 ? K : refs;
  for (int h = 0; h < hyp_total; h++) { hyp_k0[h] = -1; hyp_W[h] = 0.0; hyp_nin[h] = 0; hyp_kept[h] = 0; }
  /* when exhaustive, U is still the usable list in index order */
  double** wkeep = (double**)malloc(sizeof(double*) * (nh ? nh : 1));
  for (int h = 0; h < nh; h++) {
    int k0 = U[h];
    hyp_k0[h] = k0;
    wkeep[h] = (double*)malloc(sizeof(double) * (K ? K : 1));
    /* Eq. (2): coordinates relative to the reference, for both point sets */
    for (int k = 0; k < K; k++)
      for (int c = 0; c < 3; c++) {
        S1[3 * k + c] = o1[3 * k + c] - o1[3 * k0 + c];
        S2[3 * k + c] = o2[3 * k + c] - o2[3 * k0 + c];
      }
    for (int k = 0; k < K; k++) w[k] = usable[k] ? 1.0 : 0.0;
    int degenerate = 0;
    for (int it = 0; it < iters; it++) {
      /* R-step, Eq. (3): rotation that best maps the weighted S1 onto S2 */
      double Mx[9] = {0}, R[9];
      for (int k = 0; k < K; k++) {
        if (!usable[k]) continue;
        for (int r = 0; r < 3; r++)
          for (int c = 0; c < 3; c++) Mx[3 * r + c] += w[k] * S2[3 * k + r] * S1[3 * k + c];
      }
      if (tto_rotation_fit(Mx, R, NULL)) { degenerate = 1; break; }
      /* w-step, Eq. (4): d_k = |S2(k) - R S1(k)|, w_k = min(H / d_k, 1) (w_k = 1 at d_k = 0) */
      for (int k = 0; k < K; k++) {
        if (!usable[k]) { d[k] = INFINITY; w[k] = 0.0; continue; }
        double e[3];
        for (int r = 0; r < 3; r++)
          e[r] = S2[3 * k + r] - (R[3 * r] * S1[3 * k] + R[3 * r + 1] * S1[3 * k + 1] + R[3 * r + 2] * S1[3 * k + 2]);
        d[k] = norm3(e);
        w[k] = (d[k] > H) ? H / d[k] : 1.0;
      }
    }
    if (degenerate) {
      hyp_kept[h] = 2;
      continue;
    }
    double Wsum = 0.0;
    int nin = 0;
    for (int k = 0; k < K; k++) {
      if (!usable[k]) continue;
      Wsum += w[k];
      if (d[k] <= H) nin++;
    }
    hyp_W[h] = Wsum;
    hyp_nin[h] = nin;
    memcpy(wkeep[h], w, sizeof(double) * K);
  }
  /* a small sum of weights marks the reference as a likely outlier: keep the hypotheses whose
   * sum reaches half of the best one */
  double Wmax = 0.0;
  for (int h = 0; h < nh; h++)
    if (hyp_kept[h] != 2 && hyp_W[h] > Wmax) Wmax = hyp_W[h];
  for (int h = 0; h < nh; h++) {
    if (hyp_kept[h] == 2) continue;
    if (hyp_W[h] >= 0.5 * Wmax) {
      hyp_kept[h] = 1;
      for (int k = 0; k < K; k++)
        if (wkeep[h][k] > wstar[k]) wstar[k] = wkeep[h][k];
    }
  }
  for (int k = 0; k < K; k++) preselected[k] = (usable[k] && wstar[k] >= 0.5) ? 1 : 0;
  for (int h = 0; h < nh; h++) free(wkeep[h]);
  free(wkeep); free(U); free(w); free(d); free(S1); free(S2);
  return nh;
}

/* ------------------------------------------------------------------------------------------ */
/* Per-frame set-up                                                                            */

int tto_frame_begin(tto_stream* s, const float* depth_mm, const float* feat_xyz,
                    const uint8_t* feat_desc, int K2) {
  if (!s) return TTO_EINVAL;
  if (!s->has_template) return TTO_ESTATE;
  if (!depth_mm || K2 < 0 || (K2 > 0 && (!feat_xyz || !feat_desc))) return TTO_EINVAL;
  free_frame(s);
  int HW = s->K.width * s->K.height, K1 = s->K1, K1a = K1 ? K1 : 1;
  s->normals = (double*)malloc(sizeof(double) * 3 * HW);
  s->nvalid = (uint8_t*)malloc(HW);
  s->qpts = (double*)malloc(sizeof(double) * 3 * HW);
  s->midx = (int32_t*)malloc(sizeof(int32_t) * K1a);
  s->mdist = (int32_t*)malloc(sizeof(int32_t) * K1a);
  s->o2 = (double*)malloc(sizeof(double) * 3 * K1a);
  s->usable = (uint8_t*)malloc(K1a);
  s->wstar = (double*)malloc(sizeof(double) * K1a);
  s->presel = (uint8_t*)malloc(K1a);
  if (!s->normals || !s->nvalid || !s->qpts || !s->midx || !s->mdist || !s->o2 || !s->usable ||
      !s->wstar || !s->presel) {
    free_frame(s);
    return TTO_ENOMEM;
  }
  tto_normal_map(depth_mm, &s->K, s->normals, s->nvalid);
  for (int v = 0; v < s->K.height; v++)
    for (int u = 0; u < s->K.width; u++) {
      int pix = v * s->K.width + u;
      if (depth_ok(depth_mm[pix])) backproject(&s->K, u, v, depth_mm[pix], s->qpts + 3 * pix);
      else s->qpts[3 * pix] = s->qpts[3 * pix + 1] = s->qpts[3 * pix + 2] = 0.0;
    }
  if (K2 > 0) {
    tto_hamming_match(s->desc1, K1, feat_desc, K2, s->midx, s->mdist);
  } else {
    for (int k = 0; k < K1; k++) { s->midx[k] = -1; s->mdist[k] = 256; }
  }
  for (int k = 0; k < K1; k++) {
    int b = s->midx[k];
    s->usable[k] = 0;
    s->o2[3 * k] = s->o2[3 * k + 1] = s->o2[3 * k + 2] = 0.0;
    if (b < 0 || s->mdist[k] > s->P.max_hamming) continue;
    if (!all_finite3f(feat_xyz + 3 * b)) continue;
    for (int c = 0; c < 3; c++) s->o2[3 * k + c] = (double)feat_xyz[3 * b + c];
    s->usable[k] = 1;
  }
  tto_preselect(s->f1, s->o2, s->usable, K1, s->P.H, s->P.ransac_refs, s->P.ransac_iters, s->P.seed,
                s->frame, s->wstar, s->presel, s->hyp_k0, s->hyp_W, s->hyp_nin, s->hyp_kept);
  s->frame_ready = 1;
  return TTO_OK;
}

/* ------------------------------------------------------------------------------------------ */
/* Cost of Eq. (1) and its linearisation                                                       */

typedef struct {
  int32_t* corr;   /* [M] pixel or -1 */
  double* omega;   /* [M] Tukey weight */
  double* r_icp;   /* [M] point-to-plane residual at the association state */
  double* orbw;    /* [K1] feature weight */
  double w_arap;
  int32_t* zwin;   /* [H*W] z-buffer: the point nearest the camera at each pixel, -1 (z-buffer mode) */
  float* zmin;     /* [H*W] its z */
} assoc_t;

static int assoc_alloc(const tto_stream* s, assoc_t* a) {
  int M = s->M, K1a = s->K1 ? s->K1 : 1;
  a->corr = (int32_t*)malloc(sizeof(int32_t) * M);
  a->omega = (double*)malloc(sizeof(double) * M);
  a->r_icp = (double*)malloc(sizeof(double) * M);
  a->orbw = (double*)malloc(sizeof(double) * K1a);
  a->w_arap = 0.0;
  a->zwin = NULL;
  a->zmin = NULL;
  if (s->P.assoc_zbuffer) {
    size_t HW = (size_t)s->K.width * s->K.height;
    a->zwin = (int32_t*)malloc(sizeof(int32_t) * HW);
    a->zmin = (float*)malloc(sizeof(float) * HW);
    if (!a->zwin || !a->zmin) return -1;
  }
  return (a->corr && a->omega && a->r_icp && a->orbw) ? 0 : -1;
}
static void assoc_free(assoc_t* a) {
  free(a->corr); free(a->omega); free(a->r_icp); free(a->orbw); free(a->zwin); free(a->zmin);
}

/* Nearest pixel of a camera-frame point, u = floor(fx x / z + cx + 1/2) (same for v), or -1 if
 * z <= 0 or the pixel is outside the image. */
static int nearest_pixel(const tto_intrinsics* K, const double* v) {
  if (!(v[2] > 0.0)) return -1;
  double uf = K->fx * v[0] / v[2] + K->cx;
  double vf = K->fy * v[1] / v[2] + K->cy;
  double ur = floor(uf + 0.5), vr = floor(vf + 0.5);
  if (!(ur >= 0.0 && ur < (double)K->width && vr >= 0.0 && vr < (double)K->height)) return -1;
  return (int)vr * K->width + (int)ur;
}

/* The closest-point alternative to re-projection (Sec. 2 names closest-point search in a kd-tree as
 * the slower option): the pixel whose back-projected target point is nearest to v in 3D, over the
 * pixels that have a normal (exhaustive search, FP64 squared distance, ties to the lower pixel
 * index), or -1 if no pixel has one. */
static int nearest_point(const tto_stream* s, const double* v) {
  size_t HW = (size_t)s->K.width * s->K.height;
  double best = INFINITY;
  int arg = -1;
  for (size_t p = 0; p < HW; p++) {
    if (!s->nvalid[p]) continue;
    const double* q = s->qpts + 3 * p;
    double d[3] = {v[0] - q[0], v[1] - q[1], v[2] - q[2]};
    double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (d2 < best) { best = d2; arg = (int)p; } /* equal: the lower index, found first, stays */
  }
  return arg;
}

/* current node positions p_i^t = W_i^t(p_i^0) */
static void node_positions(const tto_stream* s, const double* dq, double* pos) {
  for (int i = 0; i < s->N; i++) dq_apply(dq + 8 * i, s->c0 + 3 * i, pos + 3 * i);
}

/* Projective association (Sec. 2): each deformed template point is re-projected to the
 * nearest pixel, u = floor(fx x / z + cx + 1/2), and corresponds to the target point there if
 * z > 0, the pixel is inside the image and it has a valid normal. The residual is the
 * point-to-plane distance along the target normal; Tukey's biweight gives its weight.
 * Feature weights (Sec. 2.1, last paragraph): pre-selected matches keep their pre-selection
 * weight; the others get clamp(1 - d_k / (5H), 0, 1) with d_k the current 3D distance.
 * The ARAP weight is scaled by the summed data weights (Sec. 2, after Eq. (1)). */
static void associate(const tto_stream* s, const double* dq, assoc_t* a, int set_warap) {
  const tto_intrinsics* K = &s->K;
  int kk = s->kk;
  double sumw = 0.0;
  if (a->zwin) {
    /* z-buffer ("rasterization", Sec. 2): a pixel belongs to the template point nearest the
     * camera among those that project to it */
    size_t HW = (size_t)K->width * K->height;
    for (size_t p = 0; p < HW; p++) { a->zwin[p] = -1; a->zmin[p] = INFINITY; }
    for (int j = 0; j < s->M; j++) {
      double v[3];
      tto_dqb(dq, s->knn_pts + kk * j, s->alpha_pts + kk * j, kk, s->pts + 3 * j, v);
      int pix = nearest_pixel(K, v);
      if (pix < 0) continue;
      float z = (float)v[2];
      if (z < a->zmin[pix]) { a->zmin[pix] = z; a->zwin[pix] = j; } /* equal z: lower j kept */
    }
  }
  for (int j = 0; j < s->M; j++) {
    double v[3];
    tto_dqb(dq, s->knn_pts + kk * j, s->alpha_pts + kk * j, kk, s->pts + 3 * j, v);
    a->corr[j] = -1;
    a->omega[j] = 0.0;
    a->r_icp[j] = 0.0;
    int pix = s->P.assoc_kdtree ? nearest_point(s, v) : nearest_pixel(K, v);
    if (pix < 0) continue;
    if (a->zwin && a->zwin[pix] != j) continue; /* hidden behind another template point */
    if (!s->nvalid[pix]) continue;
    const double* n = s->normals + 3 * pix;
    const double* q = s->qpts + 3 * pix;
    double dv[3] = {v[0] - q[0], v[1] - q[1], v[2] - q[2]};
    double r = dot3(n, dv);
    double om = 0.0;
    if (fabs(r) < s->P.tukey_c) {
      double t = r / s->P.tukey_c;
      om = (1.0 - t * t) * (1.0 - t * t);
    }
    a->corr[j] = pix;
    a->omega[j] = om;
    a->r_icp[j] = r;
    sumw += om;
  }
  double sumo = 0.0;
  for (int k = 0; k < s->K1; k++) {
    a->orbw[k] = 0.0;
    if (!s->usable[k]) continue;
    if (s->presel[k]) {
      a->orbw[k] = s->wstar[k];
    } else {
      double f[3];
      tto_dqb(dq, s->knn_feat + kk * k, s->alpha_feat + kk * k, kk, s->f1 + 3 * k, f);
      double e[3] = {f[0] - s->o2[3 * k], f[1] - s->o2[3 * k + 1], f[2] - s->o2[3 * k + 2]};
      double dk = norm3(e);
      double wk = 1.0 - dk / (5.0 * s->P.H);
      a->orbw[k] = wk < 0.0 ? 0.0 : (wk > 1.0 ? 1.0 : wk);
    }
    sumo += a->orbw[k];
  }
  if (set_warap) {
    double sd = sumw + s->P.w_orb * sumo;
    a->w_arap = (s->s_arap > 0.0) ? s->P.lambda_arap * sd / s->s_arap : 0.0;
  }
}

int tto_num_rows(const tto_stream* s) {
  if (!s || !s->has_template) return 0;
  return s->M + 3 * s->K1 + 8 * s->N * (s->N - 1);
}

/* Residual rows (and, if J != NULL, the dense Jacobian) at warps dq with association a.
 * Row order: one ICP row per template point; three feature rows per template feature; eight
 * ARAP rows per ordered node pair (a, b), a != b, a-major: length (1), angle (3), rotation (4).
 * Rows without a term are zero. */
static void residual_rows(const tto_stream* s, const double* dq, const assoc_t* a, double* r,
                          double* J) {
  int M = s->M, K1 = s->K1, N = s->N, kk = s->kk, n = 6 * N;
  int rows = M + 3 * K1 + 8 * N * (N - 1);
  if (J) memset(J, 0, sizeof(double) * (size_t)rows * n);
  double* pos = (double*)malloc(sizeof(double) * 3 * N);
  double* Q = (double*)malloc(sizeof(double) * 48 * N);
  node_positions(s, dq, pos);
  for (int i = 0; i < N; i++) dq_increment_jac(dq + 8 * i, pos + 3 * i, Q + 48 * i);

  /* f_ICP rows: sqrt(omega_j) n . (v_j - q) */
  for (int j = 0; j < M; j++) {
    r[j] = 0.0;
    if (a->corr[j] < 0 || a->omega[j] == 0.0) continue;
    const int32_t* nodes = s->knn_pts + kk * j;
    const double* al = s->alpha_pts + kk * j;
    double b[8], sg[8], v[3];
    dq_blend(dq, nodes, al, kk, b, sg);
    dq_apply(b, s->pts + 3 * j, v);
    const double* nn = s->normals + 3 * a->corr[j];
    const double* q = s->qpts + 3 * a->corr[j];
    double sw = sqrt(a->omega[j]);
    r[j] = sw * (nn[0] * (v[0] - q[0]) + nn[1] * (v[1] - q[1]) + nn[2] * (v[2] - q[2]));
    if (!J) continue;
    double Jb[24];
    dq_apply_jac(b, s->pts + 3 * j, Jb);
    double nJ[8];
    for (int c = 0; c < 8; c++) nJ[c] = nn[0] * Jb[c] + nn[1] * Jb[8 + c] + nn[2] * Jb[16 + c];
    for (int t = 0; t < kk; t++) {
      const double* Qi = Q + 48 * nodes[t];
      for (int c = 0; c < 6; c++) {
        double acc = 0.0;
        for (int m = 0; m < 8; m++) acc += nJ[m] * Qi[m * 6 + c];
        J[(size_t)j * n + 6 * nodes[t] + c] += sw * sg[t] * al[t] * acc;
      }
    }
  }
  /* f_ORB rows: sqrt(w_ORB w_k) (DQB(o1_k) - o2_k) */
  for (int k = 0; k < K1; k++) {
    int row = M + 3 * k;
    r[row] = r[row + 1] = r[row + 2] = 0.0;
    if (!s->usable[k] || a->orbw[k] == 0.0) continue;
    const int32_t* nodes = s->knn_feat + kk * k;
    const double* al = s->alpha_feat + kk * k;
    double b[8], sg[8], f[3];
    dq_blend(dq, nodes, al, kk, b, sg);
    dq_apply(b, s->f1 + 3 * k, f);
    double sw = sqrt(s->P.w_orb * a->orbw[k]);
    for (int c = 0; c < 3; c++) r[row + c] = sw * (f[c] - s->o2[3 * k + c]);
    if (!J) continue;
    double Jb[24];
    dq_apply_jac(b, s->f1 + 3 * k, Jb);
    for (int t = 0; t < kk; t++) {
      const double* Qi = Q + 48 * nodes[t];
      for (int rr = 0; rr < 3; rr++)
        for (int c = 0; c < 6; c++) {
          double acc = 0.0;
          for (int m = 0; m < 8; m++) acc += Jb[rr * 8 + m] * Qi[m * 6 + c];
          J[(size_t)(row + rr) * n + 6 * nodes[t] + c] += sw * sg[t] * al[t] * acc;
        }
    }
  }
  /* f_ARAP rows, Eqs. (5)-(6), all ordered pairs (dense connections, Sec. 2.2).
   * length: |p_b - p_a| - |p_b^0 - p_a^0|
   * angle:  chordal form a_hat - b_hat of the angle between a = W_a(p_b^0) - p_a^t = R_a e0 and
   *         b = p_b^t - p_a^t (|a_hat - b_hat|^2 = 4 sin^2(angle / 2))
   * rotation: first four components of W_a minus those of W_b */
  int row = M + 3 * K1;
  for (int ia = 0; ia < N; ia++) {
    for (int ib = 0; ib < N; ib++) {
      if (ia == ib) continue;
      double* rr = r + row;
      for (int t = 0; t < 8; t++) rr[t] = 0.0;
      double wab = a->w_arap * arap_pair_weight(s, ia, ib);
      const double* pa = pos + 3 * ia;
      const double* pb = pos + 3 * ib;
      const double* qa = dq + 8 * ia;
      const double* qb = dq + 8 * ib;
      double e0[3], av[3], bv[3];
      for (int c = 0; c < 3; c++) {
        e0[c] = s->c0[3 * ib + c] - s->c0[3 * ia + c];
        bv[c] = pb[c] - pa[c];
      }
      qrotate(qa, e0, av);
      double la = norm3(av), lb = norm3(bv), l0 = norm3(e0);
      double sl = sqrt(wab), sa = sqrt(wab * s->P.w_angle), sr = sqrt(wab * s->P.w_rotation);
      int geo = (la > 0.0 && lb > 0.0);
      double ah[3] = {0, 0, 0}, bh[3] = {0, 0, 0};
      if (geo) {
        for (int c = 0; c < 3; c++) { ah[c] = av[c] / la; bh[c] = bv[c] / lb; }
        rr[0] = sl * (lb - l0);
        for (int c = 0; c < 3; c++) rr[1 + c] = sa * (ah[c] - bh[c]);
      }
      for (int c = 0; c < 4; c++) rr[4 + c] = sr * (qa[c] - qb[c]);
      if (J) {
        double* J0 = J + (size_t)row * n;
        int ca = 6 * ia, cb = 6 * ib;
        if (geo) {
          /* length: d/dtau_a = -b_hat, d/dtau_b = +b_hat */
          for (int c = 0; c < 3; c++) {
            J0[ca + 3 + c] = -sl * bh[c];
            J0[cb + 3 + c] = sl * bh[c];
          }
          /* angle: d a_hat/d omega_a = -[a_hat]x ; d b_hat/d b = (I - b_hat b_hat^T)/|b| */
          double Sa[9];
          skew(ah, Sa);
          for (int r3 = 0; r3 < 3; r3++) {
            double* Jr = J + (size_t)(row + 1 + r3) * n;
            for (int c = 0; c < 3; c++) {
              double Pbc = ((r3 == c) ? 1.0 : 0.0) - bh[r3] * bh[c];
              Jr[ca + c] = -sa * Sa[r3 * 3 + c];
              Jr[ca + 3 + c] = sa * Pbc / lb;
              Jr[cb + 3 + c] = -sa * Pbc / lb;
            }
          }
        }
        /* rotation: d qr/d omega = G(qr)/2 */
        double Ga[12], Gb[12];
        Gmat(qa, Ga);
        Gmat(qb, Gb);
        for (int r4 = 0; r4 < 4; r4++) {
          double* Jr = J + (size_t)(row + 4 + r4) * n;
          for (int c = 0; c < 3; c++) {
            Jr[ca + c] = sr * 0.5 * Ga[r4 * 3 + c];
            Jr[cb + c] = -sr * 0.5 * Gb[r4 * 3 + c];
          }
        }
      }
      row += 8;
    }
  }
  free(pos);
  free(Q);
}

int tto_apply_increment(const tto_stream* s, const double* dq, const double* delta, double* dq_out) {
  if (!s || !s->has_template || !dq || !delta || !dq_out) return TTO_EINVAL;
  for (int i = 0; i < s->N; i++) {
    double p[3];
    dq_apply(dq + 8 * i, s->c0 + 3 * i, p);
    double o[8];
    dq_increment(dq + 8 * i, p, delta + 6 * i, o);
    memcpy(dq_out + 8 * i, o, sizeof(o));
  }
  return TTO_OK;
}

int tto_residuals(tto_stream* s, const double* dq_eval, const double* dq_assoc, double w_arap,
                  double* r, double* J, double* w_arap_used) {
  if (!s || !dq_eval || !dq_assoc || !r) return TTO_EINVAL;
  if (!s->has_template || !s->frame_ready) return TTO_ESTATE;
  assoc_t a;
  if (assoc_alloc(s, &a)) { assoc_free(&a); return TTO_ENOMEM; }
  associate(s, dq_assoc, &a, w_arap < 0.0);
  if (w_arap >= 0.0) a.w_arap = w_arap;
  if (w_arap_used) *w_arap_used = a.w_arap;
  residual_rows(s, dq_eval, &a, r, J);
  assoc_free(&a);
  return TTO_OK;
}

/* Normal equations A = J^T J, g = J^T r, accumulated point by point, match by match and pair
 * by pair over each row group's nonzero node blocks, without materialising J. */
static void normal_equations_sparse(const tto_stream* s, const double* dq, const assoc_t* a,
                                    double* A, double* g);

int tto_normal_equations(tto_stream* s, const double* dq, double w_arap, double* A, double* g) {
  if (!s || !dq || !A || !g) return TTO_EINVAL;
  if (!s->has_template || !s->frame_ready) return TTO_ESTATE;
  assoc_t a;
  if (assoc_alloc(s, &a)) { assoc_free(&a); return TTO_ENOMEM; }
  associate(s, dq, &a, w_arap < 0.0);
  if (w_arap >= 0.0) a.w_arap = w_arap;
  normal_equations_sparse(s, dq, &a, A, g);
  assoc_free(&a);
  return TTO_OK;
}

/* ------------------------------------------------------------------------------------------ */
/* Per-row Jacobian blocks without the dense matrix (same arithmetic as residual_rows)          */

/* Accumulate the outer products of a group of `nr` rows whose nonzeros sit in the node blocks
 * listed in `blk` (nb blocks of 6 columns): Jg is nr x (6 nb) row-major, rg the residuals. */
static void accum_rows(double* A, double* g, int n, const int* blk, int nb, const double* Jg,
                       const double* rg, int nr) {
  int w = 6 * nb;
  for (int row = 0; row < nr; row++) {
    const double* Jr = Jg + row * w;
    for (int x = 0; x < w; x++) {
      if (Jr[x] == 0.0) continue;
      int cx = 6 * blk[x / 6] + x % 6;
      g[cx] += Jr[x] * rg[row];
      for (int y = 0; y < w; y++) {
        if (Jr[y] == 0.0) continue;
        int cy = 6 * blk[y / 6] + y % 6;
        A[(size_t)cx * n + cy] += Jr[x] * Jr[y];
      }
    }
  }
}

static void normal_equations_sparse(const tto_stream* s, const double* dq, const assoc_t* a,
                                    double* A, double* g) {
  int M = s->M, K1 = s->K1, N = s->N, kk = s->kk, n = 6 * N;
  memset(A, 0, sizeof(double) * (size_t)n * n);
  memset(g, 0, sizeof(double) * n);
  double* pos = (double*)malloc(sizeof(double) * 3 * N);
  double* Q = (double*)malloc(sizeof(double) * 48 * N);
  node_positions(s, dq, pos);
  for (int i = 0; i < N; i++) dq_increment_jac(dq + 8 * i, pos + 3 * i, Q + 48 * i);
  int blk[8];
  double Jg[8 * 48], rg[8];
  /* a point's blend slots may repeat a node (padding) -- merge them into one block list */
  for (int j = 0; j < M + K1; j++) {
    int isf = j >= M, idx = isf ? j - M : j;
    int nr = isf ? 3 : 1;
    if (!isf && (a->corr[idx] < 0 || a->omega[idx] == 0.0)) continue;
    if (isf && (!s->usable[idx] || a->orbw[idx] == 0.0)) continue;
    const int32_t* nodes = isf ? s->knn_feat + kk * idx : s->knn_pts + kk * idx;
    const double* al = isf ? s->alpha_feat + kk * idx : s->alpha_pts + kk * idx;
    const double* p = isf ? s->f1 + 3 * idx : s->pts + 3 * idx;
    double b[8], sg[8], v[3], Jb[24];
    dq_blend(dq, nodes, al, kk, b, sg);
    dq_apply(b, p, v);
    dq_apply_jac(b, p, Jb);
    double Jrow8[3 * 8];
    double sw;
    if (!isf) {
      const double* nn = s->normals + 3 * a->corr[idx];
      const double* q = s->qpts + 3 * a->corr[idx];
      sw = sqrt(a->omega[idx]);
      rg[0] = sw * (nn[0] * (v[0] - q[0]) + nn[1] * (v[1] - q[1]) + nn[2] * (v[2] - q[2]));
      for (int c = 0; c < 8; c++) Jrow8[c] = nn[0] * Jb[c] + nn[1] * Jb[8 + c] + nn[2] * Jb[16 + c];
    } else {
      sw = sqrt(s->P.w_orb * a->orbw[idx]);
      for (int c = 0; c < 3; c++) rg[c] = sw * (v[c] - s->o2[3 * idx + c]);
      memcpy(Jrow8, Jb, sizeof(Jb));
    }
    int nb = 0;
    int slot_blk[8];
    for (int t = 0; t < kk; t++) {
      int f = -1;
      for (int u = 0; u < nb; u++)
        if (blk[u] == nodes[t]) f = u;
      if (f < 0) { blk[nb] = nodes[t]; f = nb++; }
      slot_blk[t] = f;
    }
    memset(Jg, 0, sizeof(double) * nr * 6 * nb);
    for (int t = 0; t < kk; t++) {
      const double* Qi = Q + 48 * nodes[t];
      for (int rr = 0; rr < nr; rr++)
        for (int c = 0; c < 6; c++) {
          double acc = 0.0;
          for (int m = 0; m < 8; m++) acc += Jrow8[rr * 8 + m] * Qi[m * 6 + c];
          Jg[rr * 6 * nb + 6 * slot_blk[t] + c] += sw * sg[t] * al[t] * acc;
        }
    }
    accum_rows(A, g, n, blk, nb, Jg, rg, nr);
  }
  /* ARAP rows, same formulas as residual_rows */
  for (int ia = 0; ia < N; ia++) {
    for (int ib = 0; ib < N; ib++) {
      if (ia == ib) continue;
      double wab = a->w_arap * arap_pair_weight(s, ia, ib);
      const double* pa = pos + 3 * ia;
      const double* pb = pos + 3 * ib;
      const double* qa = dq + 8 * ia;
      const double* qb = dq + 8 * ib;
      double e0[3], av[3], bv[3];
      for (int c = 0; c < 3; c++) {
        e0[c] = s->c0[3 * ib + c] - s->c0[3 * ia + c];
        bv[c] = pb[c] - pa[c];
      }
      qrotate(qa, e0, av);
      double la = norm3(av), lb = norm3(bv), l0 = norm3(e0);
      double sl = sqrt(wab), sa = sqrt(wab * s->P.w_angle), sr = sqrt(wab * s->P.w_rotation);
      int geo = (la > 0.0 && lb > 0.0);
      blk[0] = ia;
      blk[1] = ib;
      memset(Jg, 0, sizeof(double) * 8 * 12);
      for (int t = 0; t < 8; t++) rg[t] = 0.0;
      if (geo) {
        double ah[3], bh[3], Sa[9];
        for (int c = 0; c < 3; c++) { ah[c] = av[c] / la; bh[c] = bv[c] / lb; }
        rg[0] = sl * (lb - l0);
        for (int c = 0; c < 3; c++) rg[1 + c] = sa * (ah[c] - bh[c]);
        for (int c = 0; c < 3; c++) {
          Jg[0 * 12 + 3 + c] = -sl * bh[c];
          Jg[0 * 12 + 9 + c] = sl * bh[c];
        }
        skew(ah, Sa);
        for (int r3 = 0; r3 < 3; r3++)
          for (int c = 0; c < 3; c++) {
            double Pbc = ((r3 == c) ? 1.0 : 0.0) - bh[r3] * bh[c];
            Jg[(1 + r3) * 12 + c] = -sa * Sa[r3 * 3 + c];
            Jg[(1 + r3) * 12 + 3 + c] = sa * Pbc / lb;
            Jg[(1 + r3) * 12 + 9 + c] = -sa * Pbc / lb;
          }
      }
      double Ga[12], Gb[12];
      Gmat(qa, Ga);
      Gmat(qb, Gb);
      for (int c = 0; c < 4; c++) rg[4 + c] = sr * (qa[c] - qb[c]);
      for (int r4 = 0; r4 < 4; r4++)
        for (int c = 0; c < 3; c++) {
          Jg[(4 + r4) * 12 + c] = sr * 0.5 * Ga[r4 * 3 + c];
          Jg[(4 + r4) * 12 + 6 + c] = -sr * 0.5 * Gb[r4 * 3 + c];
        }
      accum_rows(A, g, n, blk, 2, Jg, rg, 8);
    }
  }
  free(pos);
  free(Q);
}

/* ------------------------------------------------------------------------------------------ */
/* Dense Cholesky (textbook, row-oriented)                                                     */

int tto_cholesky(const double* A, int n, double* L) {
  memset(L, 0, sizeof(double) * (size_t)n * n);
  for (int i = 0; i < n; i++) {
    for (int j = 0; j <= i; j++) {
      double sum = A[(size_t)i * n + j];
      for (int k = 0; k < j; k++) sum -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
      if (i == j) {
        if (!(sum > 0.0)) return i + 1;
        L[(size_t)i * n + i] = sqrt(sum);
      } else {
        L[(size_t)i * n + j] = sum / L[(size_t)j * n + j];
      }
    }
  }
  return 0;
}

void tto_cholesky_solve(const double* L, int n, const double* b, double* x) {
  for (int i = 0; i < n; i++) {
    double sum = b[i];
    for (int k = 0; k < i; k++) sum -= L[(size_t)i * n + k] * x[k];
    x[i] = sum / L[(size_t)i * n + i];
  }
  for (int i = n - 1; i >= 0; i--) {
    double sum = x[i];
    for (int k = i + 1; k < n; k++) sum -= L[(size_t)k * n + i] * x[k];
    x[i] = sum / L[(size_t)i * n + i];
  }
}

/* ------------------------------------------------------------------------------------------ */
/* Levenberg-Marquardt over the node warps (Sec. 2)                                            */

/* Per-node step (Sec. 2, each W_i updated on its own): node i solves B_i delta_i = rhs_i with
 * B_i the 6 x 6 diagonal block of the damped normal matrix. Returns 0, or 1 if a block is not
 * positive definite. */
static int node_steps(const double* A, int n, const double* rhs, double* delta) {
  double B[36], Lb[36];
  for (int i = 0; i < n / 6; i++) {
    for (int r = 0; r < 6; r++)
      for (int c = 0; c < 6; c++) B[6 * r + c] = A[(size_t)(6 * i + r) * n + 6 * i + c];
    if (tto_cholesky(B, 6, Lb) != 0) return 1;
    tto_cholesky_solve(Lb, 6, rhs + 6 * i, delta + 6 * i);
  }
  return 0;
}

static double sumsq(const double* r, int n) {
  double e = 0.0;
  for (int i = 0; i < n; i++) e += r[i] * r[i];
  return e;
}

int tto_track_frame(tto_stream* s, const float* depth_mm, const float* feat_xyz,
                    const uint8_t* feat_desc, int K2, double* out_vertices, double* out_dq,
                    tto_frame_debug* dbg) {
  if (!s) return TTO_EINVAL;
  if (!s->has_template) return TTO_ESTATE;
  int rc = tto_frame_begin(s, depth_mm, feat_xyz, feat_desc, K2);
  if (rc) return rc;
  int M = s->M, N = s->N, K1 = s->K1, n = 6 * N, kk = s->kk;
  int rows = tto_num_rows(s);
  if (dbg) {
    if (dbg->match_idx) memcpy(dbg->match_idx, s->midx, sizeof(int32_t) * K1);
    if (dbg->match_dist) memcpy(dbg->match_dist, s->mdist, sizeof(int32_t) * K1);
    if (dbg->wstar) memcpy(dbg->wstar, s->wstar, sizeof(double) * K1);
    if (dbg->preselected) memcpy(dbg->preselected, s->presel, K1);
    int R = s->P.ransac_refs;
    if (dbg->hyp_k0) memcpy(dbg->hyp_k0, s->hyp_k0, sizeof(int32_t) * R);
    if (dbg->hyp_W) memcpy(dbg->hyp_W, s->hyp_W, sizeof(double) * R);
    if (dbg->hyp_nin) memcpy(dbg->hyp_nin, s->hyp_nin, sizeof(int32_t) * R);
    if (dbg->hyp_kept) memcpy(dbg->hyp_kept, s->hyp_kept, R);
  }
  double* A = (double*)malloc(sizeof(double) * (size_t)n * n);
  double* L = (double*)malloc(sizeof(double) * (size_t)n * n);
  double* g = (double*)malloc(sizeof(double) * n);
  double* delta = (double*)malloc(sizeof(double) * n);
  double* rhs = (double*)malloc(sizeof(double) * n);
  double* r = (double*)malloc(sizeof(double) * rows);
  double* cand = (double*)malloc(sizeof(double) * 8 * N);
  assoc_t a;
  int arc = assoc_alloc(s, &a);
  if (!A || !L || !g || !delta || !rhs || !r || !cand || arc) {
    free(A); free(L); free(g); free(delta); free(rhs); free(r); free(cand);
    assoc_free(&a);
    return TTO_ENOMEM;
  }
  double lambda = s->P.lm_lambda0;
  double w_arap = 0.0;
  for (int t = 0; t < s->P.lm_iters; t++) {
    /* re-associate at the current iterate; the ARAP weight is fixed at the first iteration */
    associate(s, s->dq, &a, t == 0);
    if (t == 0) w_arap = a.w_arap;
    a.w_arap = w_arap;
    if (dbg && dbg->w_arap_iter) dbg->w_arap_iter[t] = a.w_arap;
    residual_rows(s, s->dq, &a, r, NULL);
    double e_old = sumsq(r, rows);
    normal_equations_sparse(s, s->dq, &a, A, g);
    if (t == 0 && dbg) {
      if (dbg->corr0) memcpy(dbg->corr0, a.corr, sizeof(int32_t) * M);
      if (dbg->r0) memcpy(dbg->r0, a.r_icp, sizeof(double) * M);
      if (dbg->omega0) memcpy(dbg->omega0, a.omega, sizeof(double) * M);
      if (dbg->orbw0) memcpy(dbg->orbw0, a.orbw, sizeof(double) * K1);
      if (dbg->A0) memcpy(dbg->A0, A, sizeof(double) * (size_t)n * n);
      if (dbg->g0) memcpy(dbg->g0, g, sizeof(double) * n);
      if (dbg->w_arap) *dbg->w_arap = w_arap;
    }
    /* Marquardt damping A + lambda diag(A) + eps I, eps = 1e-12 max diag(A) */
    double dmax = 0.0;
    for (int i = 0; i < n; i++)
      if (A[(size_t)i * n + i] > dmax) dmax = A[(size_t)i * n + i];
    for (int i = 0; i < n; i++) A[(size_t)i * n + i] = A[(size_t)i * n + i] * (1.0 + lambda) + 1e-12 * dmax;
    double e_new = NAN;
    int accept = 0;
    for (int i = 0; i < n; i++) rhs[i] = -g[i];
    int fail;
    if (s->P.solver == TTO_SOLVE_NODE) {
      fail = node_steps(A, n, rhs, delta);
    } else {
      fail = tto_cholesky(A, n, L) != 0;
      if (!fail) tto_cholesky_solve(L, n, rhs, delta);
    }
    if (!fail) {
      if (t == 0 && dbg && dbg->delta0) memcpy(dbg->delta0, delta, sizeof(double) * n);
      tto_apply_increment(s, s->dq, delta, cand);
      residual_rows(s, cand, &a, r, NULL);
      e_new = sumsq(r, rows);
      accept = e_new < e_old;
    }
    if (dbg) {
      if (dbg->cost_old) dbg->cost_old[t] = e_old;
      if (dbg->cost_new) dbg->cost_new[t] = e_new;
      if (dbg->lambda) dbg->lambda[t] = lambda;
      if (dbg->accepted) dbg->accepted[t] = (uint8_t)accept;
    }
    if (accept) {
      memcpy(s->dq, cand, sizeof(double) * 8 * N);
      lambda = lambda / 10.0;
      if (lambda < 1e-10) lambda = 1e-10;
    } else {
      lambda = lambda * 10.0;
      if (lambda > 1e10) lambda = 1e10;
    }
  }
  if (out_vertices)
    for (int j = 0; j < M; j++)
      tto_dqb(s->dq, s->knn_pts + kk * j, s->alpha_pts + kk * j, kk, s->pts + 3 * j, out_vertices + 3 * j);
  if (out_dq) memcpy(out_dq, s->dq, sizeof(double) * 8 * N);
  s->frame += 1;
  free(A); free(L); free(g); free(delta); free(rhs); free(r); free(cand);
  assoc_free(&a);
  return TTO_OK;
}

/* ------------------------------------------------------------------------------------------ */
/* Uniform ORB features (Sec. 2.1)                                                             */

/* radius-3 circle, clockwise from straight up: (column, row) offsets */
static const double ORB_PI = 3.14159265358979323846;

static const int FAST_CIRCLE[16][2] = {{0, -3}, {1, -3}, {2, -2}, {3, -1}, {3, 0}, {3, 1}, {2, 2}, {1, 3},
                                       {0, 3}, {-1, 3}, {-2, 2}, {-3, 1}, {-3, 0}, {-3, -1}, {-2, -2}, {-1, -3}};

void tto_orb_default_params(tto_orb_params* p) {
  p->fast_threshold = 20;
  p->nms_radius = 1;
  p->max_features = 4096;
}

int tto_fast_response(const uint8_t* img, int W, int u, int v, int t) {
  int c = img[(size_t)v * W + u];
  int cls[16], sb = 0, sd = 0;
  for (int k = 0; k < 16; k++) {
    int x = img[(size_t)(v + FAST_CIRCLE[k][1]) * W + u + FAST_CIRCLE[k][0]];
    if (x > c + t) { cls[k] = 1; sb += x - c - t; }
    else if (x < c - t) { cls[k] = -1; sd += c - x - t; }
    else cls[k] = 0;
  }
  /* longest cyclic run of one class: walk twice around the circle */
  int best = 0;
  for (int want = -1; want <= 1; want += 2) {
    int run = 0;
    for (int k = 0; k < 32; k++) {
      run = (cls[k % 16] == want) ? run + 1 : 0;
      if (run > best) best = run;
    }
  }
  if (best < 9) return 0;
  return sb > sd ? sb : sd;
}

int tto_orb_detect(const uint8_t* img, int W, int H, const float* depth, const tto_intrinsics* K,
                   const int8_t* pattern, const tto_orb_params* p, int32_t* kp, float* xyz,
                   uint8_t* desc, int32_t* angle_bin, int32_t* count) {
  if (!img || !pattern || !p || !count || W < 1 || H < 1 || p->fast_threshold < 0 || p->nms_radius < 0 ||
      p->max_features < 0 || (depth && !K) || (p->max_features > 0 && (!kp || !desc)))
    return TTO_EINVAL;
  const int B = TTO_ORB_BORDER;
  size_t HW = (size_t)W * H;
  int32_t* R = (int32_t*)calloc(HW, sizeof(int32_t));
  int32_t* S = (int32_t*)calloc(HW, sizeof(int32_t));
  int (*rot)[256][4] = (int (*)[256][4])malloc(sizeof(int) * 30 * 256 * 4);
  if (!R || !S || !rot) { free(R); free(S); free(rot); return TTO_ENOMEM; }
  /* corner responses inside the detection region */
  for (int v = B; v < H - B; v++)
    for (int u = B; u < W - B; u++) R[(size_t)v * W + u] = tto_fast_response(img, W, u, v, p->fast_threshold);
  /* 5 x 5 box sums */
  for (int v = 2; v < H - 2; v++)
    for (int u = 2; u < W - 2; u++) {
      int acc = 0;
      for (int dy = -2; dy <= 2; dy++)
        for (int dx = -2; dx <= 2; dx++) acc += img[(size_t)(v + dy) * W + u + dx];
      S[(size_t)v * W + u] = acc;
    }
  /* the pattern rotated to each of the 30 orientation bins */
  for (int b = 0; b < 30; b++) {
    double th = 2.0 * ORB_PI * b / 30.0, cs = cos(th), sn = sin(th);
    for (int k = 0; k < 256; k++)
      for (int h = 0; h < 2; h++) {
        double x = pattern[4 * k + 2 * h], y = pattern[4 * k + 2 * h + 1];
        rot[b][k][2 * h] = (int)lround(x * cs - y * sn);
        rot[b][k][2 * h + 1] = (int)lround(x * sn + y * cs);
      }
  }
  int n = 0, total = 0;
  const int r = p->nms_radius;
  for (int v = B; v < H - B; v++)
    for (int u = B; u < W - B; u++) {
      size_t i = (size_t)v * W + u;
      int Ri = R[i];
      if (Ri <= 0) continue;
      /* kept iff no other corner in the window has a larger response (ties: lower index wins) */
      int keep = 1;
      for (int dy = -r; dy <= r && keep; dy++)
        for (int dx = -r; dx <= r; dx++) {
          int uu = u + dx, vv = v + dy;
          if ((dx == 0 && dy == 0) || uu < 0 || uu >= W || vv < 0 || vv >= H) continue;
          size_t q = (size_t)vv * W + uu;
          if (R[q] > Ri || (R[q] == Ri && q < i)) { keep = 0; break; }
        }
      if (!keep) continue;
      total++;
      if (n >= p->max_features) continue;
      kp[2 * n] = u;
      kp[2 * n + 1] = v;
      /* orientation: intensity centroid over the disc of radius 15 */
      long m10 = 0, m01 = 0;
      for (int dy = -15; dy <= 15; dy++)
        for (int dx = -15; dx <= 15; dx++) {
          if (dx * dx + dy * dy > 225) continue;
          int I = img[(size_t)(v + dy) * W + u + dx];
          m10 += (long)dx * I;
          m01 += (long)dy * I;
        }
      double th = atan2((double)m01, (double)m10);
      int bin = (int)floor(th * 30.0 / (2.0 * ORB_PI) + 0.5);
      bin = ((bin % 30) + 30) % 30;
      if (angle_bin) angle_bin[n] = bin;
      uint8_t* d = desc + 32 * (size_t)n;
      memset(d, 0, 32);
      for (int k = 0; k < 256; k++) {
        const int* q = rot[bin][k];
        int sa = S[(size_t)(v + q[1]) * W + u + q[0]];
        int sb = S[(size_t)(v + q[3]) * W + u + q[2]];
        if (sa < sb) d[k >> 3] |= (uint8_t)(1u << (k & 7));
      }
      if (xyz) {
        float z = depth ? depth[i] : NAN;
        if (depth && isfinite(z) && z > 0.0f) {
          xyz[3 * n] = (float)(((double)u - K->cx) / K->fx * (double)z);
          xyz[3 * n + 1] = (float)(((double)v - K->cy) / K->fy * (double)z);
          xyz[3 * n + 2] = z;
        } else {
          xyz[3 * n] = xyz[3 * n + 1] = xyz[3 * n + 2] = NAN;
        }
      }
      n++;
    }
  count[0] = n;
  count[1] = total;
  free(R);
  free(S);
  free(rot);
  return TTO_OK;
}
