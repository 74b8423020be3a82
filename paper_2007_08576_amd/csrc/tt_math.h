// tt_math.h -- small fixed-size algebra used by the kernels: quaternions, dual quaternions,
// dual-quaternion blending and its derivative, node-centred increments, and the FP64 rotation
// fit of the 1-point RANSAC (Horn's closed-form quaternion solution).
//
// Everything here is __host__ __device__ and branch-light so that it inlines into the kernels.
// Warps are unit dual quaternions [qr.w qr.x qr.y qr.z | qd.w qd.x qd.y qd.z] mapping
// x -> R(qr) x + 2 vec(qd conj(qr)) (Sec. 2: each control point carries a dual quaternion,
// following DynamicFusion).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#define TT_HD __host__ __device__ __forceinline__

struct f3 {
  float x, y, z;
};

TT_HD f3 mk3(float x, float y, float z) { return f3{x, y, z}; }
TT_HD f3 operator+(f3 a, f3 b) { return f3{a.x + b.x, a.y + b.y, a.z + b.z}; }
TT_HD f3 operator-(f3 a, f3 b) { return f3{a.x - b.x, a.y - b.y, a.z - b.z}; }
TT_HD f3 operator*(float s, f3 a) { return f3{s * a.x, s * a.y, s * a.z}; }
TT_HD float dot(f3 a, f3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
TT_HD f3 cross(f3 a, f3 b) {
  return f3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
TT_HD float len(f3 a) { return sqrtf(dot(a, a)); }

// ---- dual quaternions --------------------------------------------------------------------

struct dq8 {
  float v[8];
};

// Hamilton product of quaternions a, b (w, x, y, z).
TT_HD void qmul4(const float* a, const float* b, float* c) {
  float w = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
  float x = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
  float y = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
  float z = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
  c[0] = w; c[1] = x; c[2] = y; c[3] = z;
}

// Transform of p by an 8-vector b read as a (possibly unnormalised) dual quaternion:
// v = p + (2/|b_r|^2) (w u x p + u x (u x p) + w f - e u + u x f), b = (w, u | e, f).
// Equals R(b_r / |b_r|) p + 2 vec(b_d conj(b_r)) / |b_r|^2, and returns p exactly for the
// identity. Used both for a node's own warp and for a blended warp.
// The displacement v - p alone (small next to p, so residuals formed from it keep their
// relative precision in FP32).
TT_HD f3 dq_disp(const float* b, f3 p) {
  float w = b[0], e = b[4];
  f3 u = mk3(b[1], b[2], b[3]);
  f3 f = mk3(b[5], b[6], b[7]);
  float s = w * w + dot(u, u);
  f3 up = cross(u, p);
  f3 X = w * up + cross(u, up) + w * f - e * u + cross(u, f);
  return (2.0f / s) * X;
}
TT_HD f3 dq_apply(const float* b, f3 p) { return p + dq_disp(b, p); }

// Rotation part only: R(q) e for a (possibly unnormalised) quaternion q.
TT_HD f3 q_rotate(const float* q, f3 e) {
  float s = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
  f3 u = mk3(q[1], q[2], q[3]);
  f3 ue = cross(u, e);
  return e + (2.0f / s) * (q[0] * ue + cross(u, ue));
}

// dv/db (3 x 8) of dq_apply at (b, p); row-major J[r*8 + c].
TT_HD void dq_apply_jac(const float* b, f3 p, float* J) {
  float w = b[0], e = b[4];
  f3 u = mk3(b[1], b[2], b[3]);
  f3 f = mk3(b[5], b[6], b[7]);
  float s = w * w + dot(u, u);
  float is = 1.0f / s;
  f3 up = cross(u, p);
  f3 X = w * up + cross(u, up) + w * f - e * u + cross(u, f);
  f3 xs = is * X;  // X / s
  float udp = dot(u, p);
  const float pp[3] = {p.x, p.y, p.z}, uu[3] = {u.x, u.y, u.z}, ff[3] = {f.x, f.y, f.z};
  const float upp[3] = {up.x, up.y, up.z}, xss[3] = {xs.x, xs.y, xs.z};
#pragma unroll
  for (int r = 0; r < 3; r++) {
    float k = 2.0f * is;
    // dX/dw = u x p + f ; ds/dw = 2w
    J[r * 8 + 0] = k * (upp[r] + ff[r] - xss[r] * 2.0f * w);
#pragma unroll
    for (int c = 0; c < 3; c++) {
      // dX/du = -w [p]x + (u.p) I + u p^T - 2 p u^T - e I - [f]x ; ds/du = 2u
      float skp = 0.0f, skf = 0.0f;  // ([p]x)_{rc}, ([f]x)_{rc}
      if (r == 0 && c == 1) { skp = -pp[2]; skf = -ff[2]; }
      if (r == 0 && c == 2) { skp = pp[1]; skf = ff[1]; }
      if (r == 1 && c == 0) { skp = pp[2]; skf = ff[2]; }
      if (r == 1 && c == 2) { skp = -pp[0]; skf = -ff[0]; }
      if (r == 2 && c == 0) { skp = -pp[1]; skf = -ff[1]; }
      if (r == 2 && c == 1) { skp = pp[0]; skf = ff[0]; }
      float I = (r == c) ? 1.0f : 0.0f;
      float d = -w * skp + udp * I + uu[r] * pp[c] - 2.0f * pp[r] * uu[c] - e * I - skf;
      J[r * 8 + 1 + c] = k * (d - xss[r] * 2.0f * uu[c]);
      // dX/df = w I + [u]x
      float sku = 0.0f;
      if (r == 0 && c == 1) sku = -uu[2];
      if (r == 0 && c == 2) sku = uu[1];
      if (r == 1 && c == 0) sku = uu[2];
      if (r == 1 && c == 2) sku = -uu[0];
      if (r == 2 && c == 0) sku = -uu[1];
      if (r == 2 && c == 1) sku = uu[0];
      J[r * 8 + 5 + c] = k * (w * I + sku);
    }
    // dX/de = -u
    J[r * 8 + 4] = -k * uu[r];
  }
}

// G(q) = [-u^T ; w I - [u]x] (4 x 3) so that (0, a) * q = G(q) a.
TT_HD void gmat(const float* q, float* G) {
  float w = q[0], x = q[1], y = q[2], z = q[3];
  G[0] = -x; G[1] = -y; G[2] = -z;
  G[3] = w;  G[4] = z;  G[5] = -y;
  G[6] = -z; G[7] = w;  G[8] = x;
  G[9] = y;  G[10] = -x; G[11] = w;
}

// dW/dxi (8 x 6, row-major Q[r*6 + c]) of W' = Delta(xi) W at xi = 0, for the node-centred
// increment about the node position p: d qr = G(qr) d omega / 2,
// d qd = (G(qd) + G(qr) [p]x) d omega / 2 + G(qr) d tau / 2.
TT_HD void dq_increment_jac(const float* W, f3 p, float* Q) {
  float Gr[12], Gd[12];
  gmat(W, Gr);
  gmat(W + 4, Gd);
  const float S[9] = {0.0f, -p.z, p.y, p.z, 0.0f, -p.x, -p.y, p.x, 0.0f};
#pragma unroll
  for (int r = 0; r < 4; r++) {
#pragma unroll
    for (int c = 0; c < 3; c++) {
      Q[r * 6 + c] = 0.5f * Gr[r * 3 + c];
      Q[r * 6 + 3 + c] = 0.0f;
      float gs = Gr[r * 3 + 0] * S[0 * 3 + c] + Gr[r * 3 + 1] * S[1 * 3 + c] + Gr[r * 3 + 2] * S[2 * 3 + c];
      Q[(4 + r) * 6 + c] = 0.5f * (Gd[r * 3 + c] + gs);
      Q[(4 + r) * 6 + 3 + c] = 0.5f * Gr[r * 3 + c];
    }
  }
}

// W' = Delta(xi) W: rotation Exp(omega) about the node position p, then translation tau;
// renormalised (unit, qr . qd = 0) with qr.w >= 0.
TT_HD void dq_increment(const float* W, f3 p, const float* xi, float* out) {
  f3 om = mk3(xi[0], xi[1], xi[2]);
  float th = len(om);
  float k = (th > 1e-6f) ? sinf(0.5f * th) / th : 0.5f - th * th * (1.0f / 48.0f);
  float qw[4] = {cosf(0.5f * th), k * om.x, k * om.y, k * om.z};
  f3 Rp = q_rotate(qw, p);
  f3 t = p - Rp + mk3(xi[3], xi[4], xi[5]);
  float tq[4] = {0.0f, t.x, t.y, t.z};
  float Dd[4];
  qmul4(tq, qw, Dd);
#pragma unroll
  for (int c = 0; c < 4; c++) Dd[c] *= 0.5f;
  float a[4], b[4];
  qmul4(qw, W, out);
  qmul4(qw, W + 4, a);
  qmul4(Dd, W, b);
#pragma unroll
  for (int c = 0; c < 4; c++) out[4 + c] = a[c] + b[c];
  float n = sqrtf(out[0] * out[0] + out[1] * out[1] + out[2] * out[2] + out[3] * out[3]);
  float in = 1.0f / n;
#pragma unroll
  for (int c = 0; c < 8; c++) out[c] *= in;
  float rd = out[0] * out[4] + out[1] * out[5] + out[2] * out[6] + out[3] * out[7];
#pragma unroll
  for (int c = 0; c < 4; c++) out[4 + c] -= rd * out[c];
  if (out[0] < 0.0f) {
#pragma unroll
    for (int c = 0; c < 8; c++) out[c] = -out[c];
  }
}

// Blend of k = 4 node warps with weights alpha; nodes whose rotation part points away from the
// first (nearest) node's are negated so that antipodal representations do not cancel.
// sgn receives the sign used per slot.
TT_HD void dq_blend4(const float* w0, const float* w1, const float* w2, const float* w3,
                     const float* alpha, float* b, float* sgn) {
  const float* ws[4] = {w0, w1, w2, w3};
#pragma unroll
  for (int c = 0; c < 8; c++) b[c] = 0.0f;
#pragma unroll
  for (int s = 0; s < 4; s++) {
    const float* q = ws[s];
    float d = w0[0] * q[0] + w0[1] * q[1] + w0[2] * q[2] + w0[3] * q[3];
    float sg = (d < 0.0f) ? -1.0f : 1.0f;
    sgn[s] = sg;
    float a = sg * alpha[s];
#pragma unroll
    for (int c = 0; c < 8; c++) b[c] += a * q[c];
  }
}

// ---- FP64 rotation fit (1-point RANSAC, Sec. 2.1, Eq. (3)) ---------------------------------

// Cyclic Jacobi on a symmetric n x n (n <= 4) matrix in place; V receives the eigenvectors
// as columns. Fixed sweep count so that the work is bounded.
template <int n>
TT_HD void jacobi_sym(double* A, double* V) {
  for (int i = 0; i < n * n; i++) V[i] = (i % (n + 1) == 0) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 12; sweep++) {
    double off = 0.0, dg = 0.0;
    for (int p = 0; p < n; p++) {
      dg += A[p * n + p] * A[p * n + p];
      for (int q = p + 1; q < n; q++) off += A[p * n + q] * A[p * n + q];
    }
    if (off <= 1e-32 * dg || off == 0.0) break;  // off-diagonal norm at the FP64 rounding level
    for (int p = 0; p < n - 1; p++) {
      for (int q = p + 1; q < n; q++) {
        double apq = A[p * n + q];
        if (apq == 0.0) continue;
        double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; k++) {
          double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; k++) {
          double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; k++) {
          double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
      }
    }
  }
}

// Rotation R (row-major) maximising sum_k w_k b_k . (R a_k), given C[i][j] = sum_k w_k b_i a_j
// (b = target, a = source), by Horn's quaternion method: the unit quaternion is the eigenvector
// of the largest eigenvalue of the 4 x 4 symmetric matrix N built from C. N's eigenvalues are
// +-s1 +- s2 +- s3 (s_i the singular values of C, signs with the parity of det C), so with them
// sorted decreasingly s1 = (l1 + l2) / 2 and s2 = (l1 + l3) / 2. Returns 1 when s2 >= 1e-9 s1
// fails (rotation not fixed), with R = I.
//
// Vw (optional) carries an eigenvector basis from one fit to the next: when warm is set, N is first
// rotated into that basis (N' = Vw^T N Vw), where a slowly changing N is nearly diagonal and the
// sweeps stop after one or two, and the eigenvectors are rotated back; Vw then receives this fit's
// basis. The eigenvalues and the rotation agree with a cold start to rounding.
TT_HD int rotation_fit_horn(const double* C, double* R, double* Vw = nullptr, bool warm = false) {
  // S_xy = sum a_x b_y = C[y][x]
  double Sxx = C[0], Syx = C[1], Szx = C[2];
  double Sxy = C[3], Syy = C[4], Szy = C[5];
  double Sxz = C[6], Syz = C[7], Szz = C[8];
  double N[16] = {Sxx + Syy + Szz, Syz - Szy,        Szx - Sxz,        Sxy - Syx,
                  Syz - Szy,       Sxx - Syy - Szz,  Sxy + Syx,        Szx + Sxz,
                  Szx - Sxz,       Sxy + Syx,        -Sxx + Syy - Szz, Syz + Szy,
                  Sxy - Syx,       Szx + Sxz,        Syz + Szy,        -Sxx - Syy + Szz};
  double V[16];
  if (Vw && warm) {
    double T[16], Np[16], U[16];
    for (int i = 0; i < 4; i++)  // T = N Vw
      for (int j = 0; j < 4; j++)
        T[i * 4 + j] = N[i * 4 + 0] * Vw[0 * 4 + j] + N[i * 4 + 1] * Vw[1 * 4 + j] + N[i * 4 + 2] * Vw[2 * 4 + j] +
                       N[i * 4 + 3] * Vw[3 * 4 + j];
    for (int i = 0; i < 4; i++)  // N' = Vw^T T
      for (int j = 0; j < 4; j++)
        Np[i * 4 + j] = Vw[0 * 4 + i] * T[0 * 4 + j] + Vw[1 * 4 + i] * T[1 * 4 + j] + Vw[2 * 4 + i] * T[2 * 4 + j] +
                        Vw[3 * 4 + i] * T[3 * 4 + j];
    for (int i = 0; i < 4; i++)  // symmetric to rounding; make it exactly so
      for (int j = i + 1; j < 4; j++) Np[j * 4 + i] = Np[i * 4 + j];
    jacobi_sym<4>(Np, U);
    for (int i = 0; i < 4; i++)  // V = Vw U
      for (int j = 0; j < 4; j++)
        V[i * 4 + j] = Vw[i * 4 + 0] * U[0 * 4 + j] + Vw[i * 4 + 1] * U[1 * 4 + j] + Vw[i * 4 + 2] * U[2 * 4 + j] +
                       Vw[i * 4 + 3] * U[3 * 4 + j];
    for (int i = 0; i < 16; i++) N[i] = Np[i];
  } else {
    jacobi_sym<4>(N, V);
  }
  if (Vw)
    for (int i = 0; i < 16; i++) Vw[i] = V[i];
  double l[4] = {N[0], N[5], N[10], N[15]};
  int best = 0;
  for (int i = 1; i < 4; i++)
    if (l[i] > l[best]) best = i;
  // sort the eigenvalues decreasingly (4 elements)
  for (int i = 1; i < 4; i++)
    for (int k = i; k > 0 && l[k] > l[k - 1]; k--) {
      double t = l[k];
      l[k] = l[k - 1];
      l[k - 1] = t;
    }
  const double s1 = 0.5 * (l[0] + l[1]), s2 = 0.5 * (l[0] + l[2]);
  for (int i = 0; i < 9; i++) R[i] = (i % 4 == 0) ? 1.0 : 0.0;
  if (!(s1 > 0.0) || s2 < 1e-9 * s1) return 1;
  double w = V[0 * 4 + best], x = V[1 * 4 + best], y = V[2 * 4 + best], z = V[3 * 4 + best];
  double nn = 1.0 / sqrt(w * w + x * x + y * y + z * z);
  w *= nn; x *= nn; y *= nn; z *= nn;
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
  return 0;
}

// SplitMix64 step (Steele, Lea and Flood, 2014).
TT_HD unsigned long long splitmix64_next(unsigned long long* state) {
  unsigned long long z = (*state += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
