// tt_chol.hip -- dense Cholesky solve of the damped normal equations (Sec. 2: the LM step is
// obtained by a Cholesky decomposition), here of the coupled 6N x 6N system in FP32.
//
// Layout: A is row-major with leading dimension ld = npad (n rounded up to the 64-wide block),
// lower triangle only; the padding rows/columns carry an identity so no block is ragged.
// Rows npad..npad+63 form one extra "right-hand-side" row block whose first row holds b^T: the
// right-looking blocked factorisation treats it like any other row block below the diagonal,
// which leaves y = L^{-1} b in that row when the factorisation ends (the forward substitution
// comes for free). The back substitution L^T x = y then walks the block columns from the last.
//
// Per block column k:
//   k_chol_panel   every workgroup factors the 64 x 64 diagonal block in LDS (16-wide blocked,
//                  leaves in registers) and inverts the factor (2 x 2 block recursion);
//                  workgroup 0 stores L_kk and L_kk^{-1}; the others form L_ik = A_ik L_kk^{-T}
//                  as a 64x64x64 product on the matrix cores
//   k_chol_update  trailing tiles A_ij -= L_ik L_jk^T, k < j <= i (plus the right-hand-side row
//                  block), 64 x 64 tiles on the matrix cores (v_mfma_f32_16x16x4_f32)
// then one k_chol_backsolve launch: workgroup b owns block row j = nb-1-b of L^T x = y, folds in
// x_k of every later block as it is published (flag per block), and publishes x_j. Workgroups only
// wait on lower-numbered ones, which the hardware dispatches first, so the waits always end; a
// bounded spin marks the solve failed instead of waiting forever.
#include "tt_internal.h"

namespace {

constexpr int NB = TT_NB;
constexpr int LDS_LD = NB + 2;  // conflict-free for the 16 x 4 MFMA operand reads
typedef float floatx4 __attribute__((ext_vector_type(4)));

// C (64 x 64) = X Y^T for X, Y in LDS (64 x 64, leading dimension LDS_LD). Four wavefronts each
// compute a 32 x 32 quadrant as 2 x 2 MFMA 16x16x4 accumulators; acc[a][b][r] holds
// C[qr + 16a + 4 (lane/16) + r][qc + 16b + lane%16].
__device__ __forceinline__ void mma64_xyT(const float (*X)[LDS_LD], const float (*Y)[LDS_LD], floatx4 acc[2][2],
                                          int& qr, int& qc) {
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  qr = 32 * (w / 2);
  qc = 32 * (w % 2);
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int b = 0; b < 2; b++) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int li = lane % 16, lk = lane / 16;
#pragma unroll 4
  for (int kk = 0; kk < NB; kk += 4) {
    float av[2], bv[2];
#pragma unroll
    for (int a = 0; a < 2; a++) av[a] = X[qr + 16 * a + li][kk + lk];
#pragma unroll
    for (int b = 0; b < 2; b++) bv[b] = Y[qc + 16 * b + li][kk + lk];
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
      for (int b = 0; b < 2; b++) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
  }
}

// Lane broadcast of a float (the readlane builtin moves 32-bit integers: pass the bits).
__device__ __forceinline__ float readlane_f(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// In-LDS Cholesky of the 64 x 64 lower triangle L, blocked by 16: wavefront 0 factors each 16 x 16
// diagonal block with rows in registers (readlane broadcasts, no barriers), then the rows below
// are solved against it and the trailing lower triangle is updated. Returns false if a pivot is
// not positive.
__device__ bool potrf64(float (*L)[LDS_LD]) {
  const int tid = threadIdx.x;
  const int lane = tid % 64, wave = tid / 64;
  __shared__ int bad;
  if (tid == 0) bad = 0;
  __syncthreads();
#pragma unroll 1
  for (int kb = 0; kb < 4; kb++) {
    const int o = 16 * kb;
    if (wave == 0) {
      const int r = lane;
      float a[16];
#pragma unroll
      for (int c = 0; c < 16; c++) a[c] = (r < 16 && c <= r) ? L[o + r][o + c] : 0.0f;
      bool ok = true;
#pragma unroll
      for (int j = 0; j < 16; j++) {
        float djj = readlane_f(a[j], j);
        ok = ok && (djj > 0.0f);
        float ljj = sqrtf(djj);
        float lrj = a[j] / ljj;
        a[j] = (r > j) ? lrj : ((r == j) ? ljj : 0.0f);
#pragma unroll
        for (int m = j + 1; m < 16; m++) {
          float lmj = readlane_f(a[j], m);
          if (r > j && m <= r) a[m] -= a[j] * lmj;
        }
      }
      if (r < 16) {
#pragma unroll
        for (int c = 0; c < 16; c++)
          if (c <= r) L[o + r][o + c] = a[c];
      }
      if (lane == 0 && !ok) bad = 1;
    }
    __syncthreads();
    const int rows = NB - o - 16;
    if (rows == 0) break;
    // rows below: x D^T = b, forward substitution over the 16 columns, one thread per row
    if (tid < rows) {
      const int r = o + 16 + tid;
      float x[16];
#pragma unroll
      for (int c = 0; c < 16; c++) {
        float s = L[r][o + c];
#pragma unroll
        for (int m = 0; m < c; m++) s -= x[m] * L[o + c][o + m];
        x[c] = s / L[o + c][o + c];
      }
#pragma unroll
      for (int c = 0; c < 16; c++) L[r][o + c] = x[c];
    }
    __syncthreads();
    // trailing lower triangle: L[i][m] -= sum_c L[i][o+c] L[m][o+c], o+16 <= m <= i < 64
    const int base = o + 16;
    const int cnt = rows * rows;
    for (int e = tid; e < cnt; e += blockDim.x) {
      const int i = base + e / rows, m = base + e % rows;
      if (m > i) continue;
      float s = 0.0f;
#pragma unroll
      for (int c = 0; c < 16; c++) s += L[i][o + c] * L[m][o + c];
      L[i][m] -= s;
    }
    __syncthreads();
  }
  return bad == 0;
}

// Li = L^{-1} for the 64 x 64 lower-triangular L, by 2 x 2 block recursion
// [[A, 0], [C, D]]^{-1} = [[A^{-1}, 0], [-D^{-1} C A^{-1}, D^{-1}]] from 16 x 16 leaves.
__device__ void trtri64(const float (*L)[LDS_LD], float (*Li)[LDS_LD], float* T /* 32*32 */) {
  const int tid = threadIdx.x;
  for (int e = tid; e < NB * NB; e += blockDim.x) Li[e / NB][e % NB] = 0.0f;
  __syncthreads();
  {
    const int b = tid / 64, c = tid % 64;
    if (b < 4 && c < 16) {
      const int o = 16 * b;
      float x[16];
#pragma unroll
      for (int i = 0; i < 16; i++) {
        float s = (i == c) ? 1.0f : 0.0f;
#pragma unroll
        for (int m = 0; m < i; m++) s -= L[o + i][o + m] * x[m];
        x[i] = s / L[o + i][o + i];
      }
#pragma unroll
      for (int i = 0; i < 16; i++)
        if (i >= c) Li[o + i][o + c] = x[i];
    }
  }
  __syncthreads();
  // 16 -> 32: two independent blocks; T = C A^{-1}; X21 = -D^{-1} T (zeros above the diagonals
  // make the full-length sums exact)
  for (int e = tid; e < 2 * 16 * 16; e += blockDim.x) {
    const int bb = e / 256, r = (e / 16) % 16, c = e % 16, o = 32 * bb;
    float s = 0.0f;
#pragma unroll
    for (int m = 0; m < 16; m++) s += L[o + 16 + r][o + m] * Li[o + m][o + c];
    T[bb * 256 + r * 16 + c] = s;
  }
  __syncthreads();
  for (int e = tid; e < 2 * 16 * 16; e += blockDim.x) {
    const int bb = e / 256, r = (e / 16) % 16, c = e % 16, o = 32 * bb;
    float s = 0.0f;
#pragma unroll
    for (int m = 0; m < 16; m++) s += Li[o + 16 + r][o + 16 + m] * T[bb * 256 + m * 16 + c];
    Li[o + 16 + r][o + c] = -s;
  }
  __syncthreads();
  // 32 -> 64
  for (int e = tid; e < 32 * 32; e += blockDim.x) {
    const int r = e / 32, c = e % 32;
    float s = 0.0f;
#pragma unroll
    for (int m = 0; m < 32; m++) s += L[32 + r][m] * Li[m][c];
    T[r * 32 + c] = s;
  }
  __syncthreads();
  for (int e = tid; e < 32 * 32; e += blockDim.x) {
    const int r = e / 32, c = e % 32;
    float s = 0.0f;
#pragma unroll
    for (int m = 0; m < 32; m++) s += Li[32 + r][32 + m] * T[m * 32 + c];
    Li[32 + r][c] = -s;
  }
  __syncthreads();
}

__global__ __launch_bounds__(256) void k_chol_panel(float* __restrict__ A, int ld, int npad, int nb, int k,
                                                    const float* __restrict__ dscale, float* __restrict__ Linv,
                                                    LMScalars* sc) {
  __shared__ float L[NB][LDS_LD];
  __shared__ float Li[NB][LDS_LD];
  __shared__ float B[NB][LDS_LD];
  __shared__ float T[32 * 32];
  const int tid = threadIdx.x;
  const size_t dk = (size_t)(NB * k);
  const int ib = k + blockIdx.x;  // row block (== nb for the right-hand-side block)
  const size_t r0 = (ib < nb) ? (size_t)(NB * ib) : (size_t)npad;
  // block column 0 is read here for the first time: apply the equilibration D A D on the way in
  // (the right-hand-side row arrives already scaled)
  for (int e = tid; e < NB * NB; e += blockDim.x) {
    const int r = e / NB, c = e % NB;
    const float dc = (k == 0) ? dscale[dk + c] : 1.0f;
    L[r][c] = (c <= r) ? A[(dk + r) * ld + dk + c] * ((k == 0) ? dscale[dk + r] * dc : 1.0f) : 0.0f;
    if (blockIdx.x > 0) {
      const float s = (k == 0 && ib < nb) ? dscale[r0 + r] * dc : 1.0f;
      B[r][c] = A[(r0 + r) * ld + dk + c] * s;
    }
  }
  __syncthreads();
  const bool ok = potrf64(L);
  if (blockIdx.x == 0 && tid == 0 && !ok) sc->chol_fail = 1;
  trtri64(L, Li, T);
  if (blockIdx.x == 0) {
    for (int e = tid; e < NB * NB; e += blockDim.x) {
      const int r = e / NB, c = e % NB;
      if (c <= r) A[(dk + r) * ld + dk + c] = L[r][c];
      Linv[(size_t)k * NB * NB + e] = Li[r][c];
    }
    return;
  }
  // L_ik = A_ik L_kk^{-T}: C[r][c] = sum_m B[r][m] Li[c][m]
  floatx4 acc[2][2];
  int qr, qc;
  mma64_xyT(B, Li, acc, qr, qc);
  const int lane = tid % 64;
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int b = 0; b < 2; b++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int row = qr + 16 * a + 4 * (lane / 16) + r, col = qc + 16 * b + lane % 16;
        A[(r0 + row) * ld + dk + col] = acc[a][b][r];
      }
}

// trailing update A_ij -= L_ik L_jk^T over 64 x 64 tiles
__global__ __launch_bounds__(256) void k_chol_update(float* __restrict__ A, int ld, int npad, int nb, int k,
                                                     const float* __restrict__ dscale) {
  __shared__ float Si[NB][LDS_LD];
  __shared__ float Sj[NB][LDS_LD];
  const int m = nb - 1 - k;  // trailing block columns
  const int tri = m * (m + 1) / 2;
  const int t = blockIdx.x;
  int ii, jj;
  if (t < tri) {
    ii = (int)((sqrtf(8.0f * t + 1.0f) - 1.0f) * 0.5f);
    while ((ii + 1) * (ii + 2) / 2 <= t) ii++;
    while (ii * (ii + 1) / 2 > t) ii--;
    jj = t - ii * (ii + 1) / 2;
  } else {
    ii = m;  // right-hand-side block
    jj = t - tri;
  }
  const int bi = k + 1 + ii, bj = k + 1 + jj;
  const size_t ri = (bi < nb) ? (size_t)(NB * bi) : (size_t)npad;
  const size_t rj = (size_t)(NB * bj);
  const size_t ck = (size_t)(NB * k);
  const int tid = threadIdx.x;
  for (int e = tid; e < NB * NB / 4; e += 256) {
    const int r = e / (NB / 4), c4 = (e % (NB / 4)) * 4;
    const float4 a = *reinterpret_cast<const float4*>(A + (ri + r) * ld + ck + c4);
    const float4 b = *reinterpret_cast<const float4*>(A + (rj + r) * ld + ck + c4);
    Si[r][c4] = a.x; Si[r][c4 + 1] = a.y; Si[r][c4 + 2] = a.z; Si[r][c4 + 3] = a.w;
    Sj[r][c4] = b.x; Sj[r][c4 + 1] = b.y; Sj[r][c4 + 2] = b.z; Sj[r][c4 + 3] = b.w;
  }
  __syncthreads();
  floatx4 acc[2][2];
  int qr, qc;
  mma64_xyT(Si, Sj, acc, qr, qc);
  const int lane = tid % 64;
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int b = 0; b < 2; b++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const size_t row = ri + qr + 16 * a + 4 * (lane / 16) + r;
        const size_t c = rj + qc + 16 * b + lane % 16;
        // step 0 is the first touch of every trailing tile: equilibrate it (not the rhs row)
        const float s = (k == 0 && bi < nb) ? dscale[row] * dscale[c] : 1.0f;
        A[row * ld + c] = A[row * ld + c] * s - acc[a][b][r];
      }
}

constexpr long long kSpinLimit = 1ll << 22;

__device__ __forceinline__ bool wait_flag(const int* flag, int epoch) {
  long long spins = 0;
  while (__hip_atomic_load(flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
    if (++spins > kSpinLimit) return false;
    __builtin_amdgcn_s_sleep(1);
  }
  return true;
}

// Back substitution L^T x = y (y in the right-hand-side row): one wavefront per block row.
__global__ __launch_bounds__(64) void k_chol_backsolve(const float* __restrict__ A, int ld, int npad, int nb,
                                                      const float* __restrict__ Linv, float* __restrict__ x,
                                                      int* __restrict__ flags, int epoch, LMScalars* sc) {
  __shared__ float xs[NB];
  __shared__ float rs[NB];
  const int j = nb - 1 - (int)blockIdx.x;
  const int c = threadIdx.x;
  const float* yrow = A + (size_t)npad * ld;
  float acc = 0.0f;
  bool ok = true;
  for (int k = nb - 1; k > j; k--) {
    // the tile column is ready (written by the factorisation); load it before waiting
    float col[NB];
#pragma unroll
    for (int m = 0; m < NB; m++) col[m] = A[(size_t)(NB * k + m) * ld + NB * j + c];
    if (c == 0) ok = wait_flag(flags + k, epoch) && ok;
    __syncthreads();
    __threadfence();
    xs[c] = __hip_atomic_load(x + NB * k + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
#pragma unroll
    for (int m = 0; m < NB; m++) acc += col[m] * xs[m];
    __syncthreads();
  }
  rs[c] = yrow[NB * j + c] - acc;
  __syncthreads();
  const float* Li = Linv + (size_t)j * NB * NB;
  float s = 0.0f;
#pragma unroll 8
  for (int m = 0; m < NB; m++) s += Li[m * NB + c] * rs[m];
  __hip_atomic_store(x + NB * j + c, s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  if (c == 0) {
    __threadfence();
    __hip_atomic_store(flags + j, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    if (!ok) sc->chol_fail = 1;
  }
}

}  // namespace

hipError_t launch_cholesky_solve(DevState& d, int epoch, hipStream_t st) {
  const int nb = d.nb;
  for (int k = 0; k < nb; k++) {
    hipLaunchKernelGGL(k_chol_panel, dim3(nb - k + 1), dim3(256), 0, st, d.A, d.ld, d.npad, nb, k, d.dscale, d.Linv,
                       d.sc);
    const int m = nb - 1 - k;
    const int tiles = m * (m + 1) / 2 + m;
    if (tiles > 0)
      hipLaunchKernelGGL(k_chol_update, dim3(tiles), dim3(256), 0, st, d.A, d.ld, d.npad, nb, k, d.dscale);
  }
  hipLaunchKernelGGL(k_chol_backsolve, dim3(nb), dim3(64), 0, st, d.A, d.ld, d.npad, nb, d.Linv, d.x, d.flags,
                     epoch, d.sc);
  return hipGetLastError();
}
