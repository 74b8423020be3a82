// tt_chol.hip -- dense Cholesky solve of the damped normal equations (Sec. 2: the LM step is
// obtained by a Cholesky decomposition), here of the coupled 6N x 6N system in FP32.
//
// Layout: A is row-major with leading dimension ld = npad (n rounded up to the 64-wide block),
// lower triangle only; the padding rows/columns carry an identity so no block is ragged.
// Rows npad..npad+63 form one extra "right-hand-side" row block whose first row holds b^T: the
// blocked factorisation treats it like any other row block below the diagonal, which leaves
// y = L^{-1} b in that row when the factorisation ends (the forward substitution comes for free).
// The back substitution L^T x = y then walks the block columns from the last.
//
// k_chol_dataflow factors the whole matrix in one persistent launch (tile tasks with flags, see
// below); 64 x 64 x 64 tile products run on the matrix cores (v_mfma_f32_16x16x4_f32) and the
// diagonal blocks are factored and inverted inside one workgroup. Then one k_chol_backsolve
// launch: workgroup b owns block row j = nb-1-b of L^T x = y, folds in x_k of every later block as
// it is published (flag per block), and publishes x_j. Workgroups only wait on lower-numbered
// ones, which the hardware dispatches first, so the waits always end; a bounded spin marks the
// solve failed instead of waiting forever.
#include "tt_internal.h"

namespace {

// Hand-over between workgroups (possibly on different XCDs, each with its own L2) through memory.
// Every store of hand-over data (tiles, partial tiles, inverse blocks) is device-coherent (sc1): it
// writes through the L2 to memory, so a publication waits only for its own workgroup's stores
// (s_waitcnt, then the barrier) before it stores the flag, and no write-back of the whole L2 sits on
// the critical path. The consumer polls the flag, invalidates its caches (stale copies of a tile's
// lines that its XCD read or wrote earlier) and waits for the invalidation before any wavefront
// reads the tile. That wait is explicit: the compiler's own wait after the fence is dropped when no
// load or store is outstanding before it, and a load racing the invalidation can hit a stale line.
__device__ __forceinline__ void acquire_done() {
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  __builtin_amdgcn_s_waitcnt(0);
}
__device__ __forceinline__ void st_coh(float* p, float v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coh16(uint16_t* p, uint16_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Four consecutive floats (16-byte aligned) written through to memory in one instruction (the
// trailing s_nop keeps the data registers unchanged for the cycle after the store reads them).
__device__ __forceinline__ void st_coh4(float* p, float4 v) {
  typedef float v4f __attribute__((ext_vector_type(4)));
  const v4f d = {v.x, v.y, v.z, v.w};
  asm volatile("global_store_dwordx4 %0, %1, off sc1\n\ts_nop 1" : : "v"(p), "v"(d) : "memory");
}
__device__ __forceinline__ void st_coh16x4(uint16_t* p, uint64_t v) {  // four 16-bit values, 8-byte aligned
  __hip_atomic_store(reinterpret_cast<uint64_t*>(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// The calling thread's device-coherent stores (and, after a barrier, the workgroup's) are complete
// when the flag is stored.
__device__ __forceinline__ void publish_flag(int* f, int v) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_waitcnt(0);
  __hip_atomic_store(f, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr int NB = TT_NB;
constexpr int LDS_LD = NB + 2;  // conflict-free for the 16 x 4 MFMA operand reads
typedef float floatx4 __attribute__((ext_vector_type(4)));
// Eight 16-bit values as a native vector: copies of it are plain register moves (HIP's uint4 is a
// struct copied by memcpy, which keeps arrays of it in private memory).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

#define MFMA16(a, b, c) __builtin_amdgcn_mfma_f32_16x16x4f32((a), (b), (c), 0, 0, 0)

// Row broadcasts (DPP row_newbcast: lane n of each 16-lane row feeds the whole row; a VALU operand
// modifier, no LDS traffic). n must fold to a constant (the callers' loops are fully unrolled).
// Written as inline assembly so that the broadcast and the multiply-add are one v_fmac_f32_dpp; the
// leading s_nop gives the two wait states a DPP source needs after a VALU write to it.
__device__ __forceinline__ void fmac_bcast16(float& acc, float src, float mul, int n, bool guard) {
  // acc += (src of lane n of the row) * mul
  if (guard) {
    switch (n) {
    case 0: asm("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 row_newbcast:0 row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(src), "v"(mul)); break;
    case 1: asm("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 row_newbcast:1 row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(src), "v"(mul)); break;
    case 2: asm("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 row_newbcast:2 row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(src), "v"(mul)); break;
    case 3: asm("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 row_newbcast:3 row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(src), "v"(mul)); break;
    case 4: asm("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 row_newbcast:4 row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(src), "v"(mul)); break;
    case 5: asm("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 row_newbcast:5 row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(src), "v"(mul)); break;
    case 6: asm("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 row_newbcast:6 row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(src), "v"(mul)); break;
    case 7: asm("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 row_newbcast:7 row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(src), "v"(mul)); break;
    case 8: asm("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 row_newbcast:8 row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(src), "v"(mul)); break;
    case 9: asm("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 row_newbcast:9 row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(src), "v"(mul)); break;
    case 10: asm("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 row_newbcast:10 row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(src), "v"(mul)); break;
    case 11: asm("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 row_newbcast:11 row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(src), "v"(mul)); break;
    case 12: asm("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 row_newbcast:12 row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(src), "v"(mul)); break;
    case 13: asm("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 row_newbcast:13 row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(src), "v"(mul)); break;
    case 14: asm("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 row_newbcast:14 row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(src), "v"(mul)); break;
    case 15: asm("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 row_newbcast:15 row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(src), "v"(mul)); break;
    }
  } else {
    switch (n) {
    case 0: asm("v_fmac_f32_dpp %0, %1, %2 row_newbcast:0 row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(src), "v"(mul)); break;
    case 1: asm("v_fmac_f32_dpp %0, %1, %2 row_newbcast:1 row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(src), "v"(mul)); break;
    case 2: asm("v_fmac_f32_dpp %0, %1, %2 row_newbcast:2 row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(src), "v"(mul)); break;
    case 3: asm("v_fmac_f32_dpp %0, %1, %2 row_newbcast:3 row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(src), "v"(mul)); break;
    case 4: asm("v_fmac_f32_dpp %0, %1, %2 row_newbcast:4 row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(src), "v"(mul)); break;
    case 5: asm("v_fmac_f32_dpp %0, %1, %2 row_newbcast:5 row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(src), "v"(mul)); break;
    case 6: asm("v_fmac_f32_dpp %0, %1, %2 row_newbcast:6 row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(src), "v"(mul)); break;
    case 7: asm("v_fmac_f32_dpp %0, %1, %2 row_newbcast:7 row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(src), "v"(mul)); break;
    case 8: asm("v_fmac_f32_dpp %0, %1, %2 row_newbcast:8 row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(src), "v"(mul)); break;
    case 9: asm("v_fmac_f32_dpp %0, %1, %2 row_newbcast:9 row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(src), "v"(mul)); break;
    case 10: asm("v_fmac_f32_dpp %0, %1, %2 row_newbcast:10 row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(src), "v"(mul)); break;
    case 11: asm("v_fmac_f32_dpp %0, %1, %2 row_newbcast:11 row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(src), "v"(mul)); break;
    case 12: asm("v_fmac_f32_dpp %0, %1, %2 row_newbcast:12 row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(src), "v"(mul)); break;
    case 13: asm("v_fmac_f32_dpp %0, %1, %2 row_newbcast:13 row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(src), "v"(mul)); break;
    case 14: asm("v_fmac_f32_dpp %0, %1, %2 row_newbcast:14 row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(src), "v"(mul)); break;
    case 15: asm("v_fmac_f32_dpp %0, %1, %2 row_newbcast:15 row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(src), "v"(mul)); break;
    }
  }
}

// (src of lane n of the row) * m and -(src of lane n of the row) * m as one v_mul_f32_dpp each; the
// leading s_nop covers a VALU write of src just before. mul_bcast16_fenced adds a trailing s_nop so
// that its result may be the broadcast source of whichever instruction the compiler puts next.
#define TT_BC16_CASES(X) X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15)
__device__ __forceinline__ float mul_bcast16(float src, float m, int n) {
  float d;
  switch (n) {
#define TT_C(k) case k: asm("s_nop 1\n\tv_mul_f32_dpp %0, %1, %2 row_newbcast:" #k " row_mask:0xf bank_mask:0xf" : "=v"(d) : "v"(src), "v"(m)); break;
    TT_BC16_CASES(TT_C)
#undef TT_C
  }
  return d;
}
__device__ __forceinline__ float mul_bcast16_fenced(float src, float m, int n) {
  float d;
  switch (n) {
#define TT_C(k) case k: asm("s_nop 1\n\tv_mul_f32_dpp %0, %1, %2 row_newbcast:" #k " row_mask:0xf bank_mask:0xf\n\ts_nop 1" : "=v"(d) : "v"(src), "v"(m)); break;
    TT_BC16_CASES(TT_C)
#undef TT_C
  }
  return d;
}
__device__ __forceinline__ float nmul_bcast16(float src, float m, int n) {
  float d;
  switch (n) {
#define TT_C(k) case k: asm("s_nop 1\n\tv_mul_f32_dpp %0, -%1, %2 row_newbcast:" #k " row_mask:0xf bank_mask:0xf" : "=v"(d) : "v"(src), "v"(m)); break;
    TT_BC16_CASES(TT_C)
#undef TT_C
  }
  return d;
}

// 16 x 16 leaf on one wavefront: factors the block at (o, o) of L (read from LDS into registers)
// and writes the inverse of the factor to Li at (o, o); L itself is left as it was. Lane r (mod 16)
// keeps row r in registers; pivots and column entries move between lanes by row broadcasts, so
// each 16-lane row of the wave runs the same factorisation. Step j: every lane takes 1/sqrt of its
// own entry j (only lane j's, the pivot's, is used), and the broadcast of that value from lane j
// scales the column in the same instruction. The inverse is built column-oriented (lane r holds
// column r): x_i = p_i / L_ii, then p_k -= L_ki x_i for k > i.
// No lane masks: in lanes r < j, entry j and everything derived from it lie in the row's upper
// triangle, which is never broadcast (sources are lane j for the pivot and lanes m > j for the
// column) and never stored. A pivot that is not positive leaves a non-finite or non-positive
// diagonal entry of the inverse (1/sqrt of it), which the caller checks.
__device__ __forceinline__ void leaf16(float (*L)[LDS_LD], float (*Li)[LDS_LD], int o) {
  const int lane = threadIdx.x & 63, r = lane & 15;
  const bool writer = lane < 16;
  float a[16];
#pragma unroll
  for (int c = 0; c < 16; c += 2) {
    const float2 v = *reinterpret_cast<const float2*>(&L[o + r][o + c]);
    a[c] = v.x;
    a[c + 1] = v.y;
  }
  float il[16];
#pragma unroll
  for (int j = 0; j < 16; j++) {
    il[j] = __builtin_amdgcn_rsqf(a[j]);
    const float lr = mul_bcast16_fenced(il[j], a[j], j);  // the broadcast source of the updates below
    const float nlr = nmul_bcast16(il[j], a[j], j);
    a[j] = lr;
#pragma unroll
    for (int m = j + 1; m < 16; m++) fmac_bcast16(a[m], lr, nlr, m, false);
  }
  float p[16], x[16];
#pragma unroll
  for (int i = 0; i < 16; i++) p[i] = (i == r) ? 1.0f : 0.0f;
#pragma unroll
  for (int i = 0; i < 16; i++) {
    x[i] = mul_bcast16(il[i], p[i], i);
    const float nx = nmul_bcast16(il[i], p[i], i);
#pragma unroll
    for (int k = i + 1; k < 16; k++) fmac_bcast16(p[k], a[i], nx, k, k == i + 1);
  }
  if (writer) {
#pragma unroll
    for (int i = 0; i < 16; i++) Li[o + i][o + r] = (i >= r) ? x[i] : 0.0f;
  }
}

// 16 x 16 tile products on the matrix cores (v_mfma_f32_16x16x4f32), row-major tiles in LDS with
// strides given as template arguments. acc element q of lane (li, lk) = (lane % 16, lane / 16) is
// entry (4 lk + q, li).
// The operand loads of a product are all issued before its first MFMA (a scheduling barrier keeps
// the compiler from pairing each load with its MFMA, which costs one LDS round trip per MFMA when
// registers are scarce). nk = number of 16-wide reduction blocks (a compile-time value after
// unrolling at every call site).
template <int SA, int SB>
__device__ __forceinline__ floatx4 mm16_abt(const float* A, const float* B, floatx4 acc, int nk = 1) {  // acc += A B^T
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  float a[16], b[16];
#pragma unroll
  for (int t = 0; t < 16; t++)
    if (t < 4 * nk) {
      a[t] = A[li * SA + 4 * t + lk];
      b[t] = B[li * SB + 4 * t + lk];
    }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int t = 0; t < 16; t++)
    if (t < 4 * nk) acc = MFMA16(a[t], b[t], acc);
  return acc;
}
template <int SA, int SB>
__device__ __forceinline__ floatx4 mm16_ab(const float* A, const float* B, floatx4 acc) {  // acc += A B
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  float a[4], b[4];
#pragma unroll
  for (int t = 0; t < 4; t++) {
    a[t] = A[li * SA + 4 * t + lk];
    b[t] = B[(4 * t + lk) * SB + li];
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int t = 0; t < 4; t++) acc = MFMA16(a[t], b[t], acc);
  return acc;
}
template <int SC>
__device__ __forceinline__ void put16(float* C, floatx4 acc, float sign) {  // C = sign * acc
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int q = 0; q < 4; q++) C[(4 * lk + q) * SC + li] = sign * acc[q];
}
template <int SC>
__device__ __forceinline__ void sub16(float* C, floatx4 acc) {  // C -= acc
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int q = 0; q < 4; q++) C[(4 * lk + q) * SC + li] -= acc[q];
}

constexpr int XS = 18;  // stride of the 16 x 16 scratch tiles
constexpr int POTRF_SCRATCH_FLOATS = 12 * 16 * XS;

// Cholesky factor and inverse Li of the 64 x 64 lower triangle in L (LDS), blocked by 16. Writing
// T_rc for the 16 x 16 tiles of L and X_rk = T_rk Li_kk^T for the factor's off-diagonal tiles, the
// serial chain is leaf(k) -> X_{k+1,k} -> T_{k+1,k+1} -= X X^T -> leaf(k+1); wavefront 0 runs only
// that chain, while wavefronts 1-3 compute the other X tiles (each keeps its own copy of the ones it
// needs; copies of one tile are bit-identical), the trailing updates and the blocks of the inverse.
// From L Li = I, the block below the diagonal is Li_rc = -Li_rr S_rc with
// S_rc = sum_{c <= m < r} X_rm Li_mc; every S_rc is complete when leaf 3 ends, so only the three
// products Li_3c = -Li_33 S_3c follow the chain. Five barriers.
// L's off-diagonal tiles are left as the updated T (only Li is an output; its six tiles above the
// diagonal are neither read nor written and must hold zeros, which the caller sets once); scratch holds
// POTRF_SCRATCH_FLOATS floats of LDS. Returns false if a pivot is not positive (a diagonal entry
// of Li that is not positive and finite). All 256 threads must call it.
// Optionally (U non-null) the block is first updated, L -= U U^T with U the 64 x 64 tile in LDS:
// wavefront 0 updates only tile (0, 0) before leaf 0 and the others update the remaining nine lower
// tiles meanwhile. When pub is non-null, wavefronts 1-3 then run ustore() (the caller's stores of U
// to global memory); at the start of the second phase they complete those stores and the last of
// the three raises *pub = epoch (arrivals counted in the LDS word *pub_cnt, which must be 0 on entry
// and is 0 again on return); wavefront 0, on the critical path, neither stores nor waits. Scratch is first written after that phase, so U may share
// its memory. pre() runs on every thread right after the barrier that ends the fourth phase (the
// look ahead's results are in LDS by then), before the three products of the last phase.
struct NoOp {
  __device__ void operator()() const {}
};
// A look ahead that one idle thread runs during the factorisation's fourth phase: it reads the
// ticket counter into *s_ctr and whether both flags f0, f1 (if non-null) equal epoch into *s_ready,
// acquiring when they do; the results are in LDS for the whole block once the call returns. If the
// flags were not yet raised, an idle thread of the fifth phase looks again and leaves the answer in
// *s_ready2 (0 when the first look succeeded), in LDS once the factorisation returns.
struct ChainPoll {
  const int* f0;
  const int* f1;
  const int* ctr;
  int epoch;
  int* s_ready;
  int* s_ctr;
  int* s_ready2;
};
__device__ __forceinline__ void chain_poll(const ChainPoll& q) {
  const int c = __hip_atomic_load(q.ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  bool r = true;
  if (q.f0) {
    const int v0 = __hip_atomic_load(q.f0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int v1 = __hip_atomic_load(q.f1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    r = (v0 == q.epoch) && (v1 == q.epoch);
    if (r) acquire_done();
  }
  *q.s_ctr = c;
  *q.s_ready = r ? 1 : 0;
}

// One wavefront's share of a publication by n wavefronts: its device-coherent stores complete, then
// it counts itself in *cnt (LDS); the n-th to arrive resets the count and raises *flag = epoch, by
// which time every one of those wavefronts' stores has reached memory.
__device__ __forceinline__ void wave_publish(int* cnt, int* flag, int epoch, int n = 4) {
  __builtin_amdgcn_s_waitcnt(0);
  if ((threadIdx.x & 63) == 0) {
    const int prev = __hip_atomic_fetch_add(cnt, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (prev == n - 1) {
      __hip_atomic_store(cnt, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      publish_flag(flag, epoch);
    }
  }
}

template <typename UStore = NoOp, typename Pre = NoOp>
__device__ __forceinline__ bool potrf_trtri64(float (*L)[LDS_LD], float (*Li)[LDS_LD], float* scratch,
                                              const float (*U)[LDS_LD] = nullptr, int* pub = nullptr,
                                              int pub_epoch = 0, const ChainPoll* poll = nullptr,
                                              int* pub_cnt = nullptr, UStore ustore = UStore(), Pre pre = Pre()) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // scratch tiles: 0 = X10, 1 = X20, 2 = X30, 3 = X21, 4 = X31, 5 = X32, then the sums S_rc
  enum { S10 = 6, S20, S21, S30, S31, S32 };
  auto Xt = [&](int id) { return scratch + id * 16 * XS; };
  auto Lt = [&](int r, int c) { return &L[16 * r][16 * c]; };
  auto Lit = [&](int r, int c) { return &Li[16 * r][16 * c]; };
  const floatx4 z4 = {0.f, 0.f, 0.f, 0.f};
  // X_rk = T_rk Li_kk^T into scratch tile id
  auto makeX = [&](int r, int k, int id) { put16<XS>(Xt(id), mm16_abt<LDS_LD, LDS_LD>(Lt(r, k), Lit(k, k), z4), 1.0f); };
  // T_rc -= X_a X_b^T
  auto updT = [&](int r, int c, int a, int b) { sub16<LDS_LD>(Lt(r, c), mm16_abt<XS, XS>(Xt(a), Xt(b), z4)); };
  // acc += X_a Li_mc
  auto xli = [&](int a, int m, int c, floatx4 acc) { return mm16_ab<XS, LDS_LD>(Xt(a), Lit(m, c), acc); };
  // Li_rc = -Li_rr S
  auto finish = [&](int r, int c, int sid) { put16<LDS_LD>(Lit(r, c), mm16_ab<LDS_LD, XS>(Lit(r, r), Xt(sid), z4), -1.0f); };
  // T_rc -= U_r U_c^T over the 64-wide reduction (the block update folded into phase 1)
  auto updU = [&](int r, int c) {
    sub16<LDS_LD>(Lt(r, c), mm16_abt<LDS_LD, LDS_LD>(&U[16 * r][0], &U[16 * c][0], z4, NB / 16));
  };
  floatx4 s3 = z4;  // S_31 (wavefront 1) or S_30 (wavefront 2), carried from phase 3 to phase 4
  // phase 1: (update tile (0, 0)) leaf 0; the other wavefronts update the other tiles and clear
  // the upper tiles of Li
  if (wave == 0) {
    if (U) updU(0, 0);
    leaf16(L, Li, 0);
  } else {
    if (U) {
      if (wave == 1) {
        updU(1, 0);
        updU(1, 1);
        updU(2, 0);
      } else if (wave == 2) {
        updU(2, 1);
        updU(2, 2);
        updU(3, 0);
      } else {
        updU(3, 1);
        updU(3, 2);
        updU(3, 3);
      }
    }
    if (pub) ustore();
  }
  __syncthreads();
  // the stores of U were issued a phase ago: completing them and raising the flag costs little now
  if (pub && wave != 0) wave_publish(pub_cnt, pub, pub_epoch, 3);
  // phase 2: leaf 1; X_r0, trailing updates
  if (wave == 0) {
    makeX(1, 0, 0);
    updT(1, 1, 0, 0);
    leaf16(L, Li, 16);
  } else if (wave == 1) {
    makeX(1, 0, 0);
    makeX(2, 0, 1);
    updT(2, 1, 1, 0);
    updT(2, 2, 1, 1);
  } else if (wave == 2) {
    makeX(1, 0, 0);
    makeX(2, 0, 1);
    makeX(3, 0, 2);
    updT(3, 1, 2, 0);
    updT(3, 2, 2, 1);
  } else {
    makeX(3, 0, 2);
    updT(3, 3, 2, 2);
  }
  __syncthreads();
  // phase 3: leaf 2; X_r1, trailing updates; Li_10; S_21 and the first terms of S_31, S_30
  if (wave == 0) {
    makeX(2, 1, 3);
    updT(2, 2, 3, 3);
    leaf16(L, Li, 32);
  } else if (wave == 1) {
    makeX(2, 1, 3);
    makeX(3, 1, 4);
    updT(3, 2, 4, 3);
    put16<XS>(Xt(S21), xli(3, 1, 1, z4), 1.0f);
    s3 = xli(4, 1, 1, z4);
  } else if (wave == 2) {
    makeX(3, 1, 4);
    updT(3, 3, 4, 4);
    s3 = xli(2, 0, 0, z4);
  } else {
    put16<XS>(Xt(S10), xli(0, 0, 0, z4), 1.0f);
    finish(1, 0, S10);
  }
  __syncthreads();
  // phase 4: leaf 3; X_32; Li_21, Li_20; S_32 and the rest of S_31, S_30
  if (wave == 0) {
    makeX(3, 2, 5);
    updT(3, 3, 5, 5);
    leaf16(L, Li, 48);
  } else if (wave == 1) {
    makeX(3, 2, 5);
    finish(2, 1, S21);
    put16<XS>(Xt(S31), xli(5, 2, 1, s3), 1.0f);
  } else if (wave == 2) {
    put16<XS>(Xt(S20), xli(3, 1, 0, xli(1, 0, 0, z4)), 1.0f);
    finish(2, 0, S20);
    makeX(3, 2, 5);
    put16<XS>(Xt(S30), xli(5, 2, 0, xli(4, 1, 0, s3)), 1.0f);
  } else {
    makeX(3, 2, 5);
    put16<XS>(Xt(S32), xli(5, 2, 2, z4), 1.0f);
    if (poll && lane == 0) chain_poll(*poll);
  }
  __syncthreads();
  pre();
  // phase 5: Li_3c = -Li_33 S_3c
  if (wave == 1) {
    finish(3, 1, S31);
  } else if (wave == 2) {
    finish(3, 0, S30);
  } else if (wave == 3) {
    finish(3, 2, S32);
  } else if (poll && lane == 0) {
    int r2 = 0;
    if (!*poll->s_ready) {
      ChainPoll q = *poll;
      q.s_ready = &r2;
      chain_poll(q);
    }
    *poll->s_ready2 = r2;
  }
  __syncthreads();
  // every wavefront checks all 64 diagonal entries of the inverse (1 / the pivots' square roots)
  const float dv = Li[lane][lane];
  return __all((dv > 0.0f) && (dv < __builtin_huge_valf()));
}

// ---- dataflow factorisation: one persistent launch per solve ---------------------------------
//
// Left-looking tile tasks, handed out in a fixed order through an atomic ticket counter. Task
// kinds, for block column c (tiles are 64 x 64; row block nb is the right-hand side):
//   CRIT(j)      the critical chain: L_{j,j-1} = C_{j,j-1} Linv_{j-1}^T, C_jj -= L_{j,j-1} L_{j,j-1}^T,
//                then factor and invert C_jj (publishes L_{j,j-1} and Linv_j); all CRIT steps run
//                on one workgroup, which keeps Linv_j in LDS from one step to the next
//   DIAGP(j)     C_jj = A_jj - sum_{k <= j-2} L_jk L_jk^T            (j >= 2; finished by CRIT(j))
//   SUBP(j)      C_{j,j-1} = A_{j,j-1} - sum_{k <= j-2} L_jk L_{j-1,k}^T  (j >= 2; finished by CRIT(j)).
//                The last term does not wait for the chain: L_{j-1,j-2} = C_{j-1,j-2} Linv_{j-2}^T is
//                formed here again from SUBP(j-1)'s tile and Linv_{j-2}, so SUBP(j) is ready while
//                CRIT(j-1) is still factoring (for j = 2 the term L_{1,0} is read once CRIT(1) has
//                published it: CRIT(1) overwrites the raw A_{1,0} it would be formed from). C_{j,j-1} is kept in the unused upper-triangle tile
//                (j-1, j) of A, so that CRIT(j) can overwrite tile (j, j-1) with L while SUBP(j+1)
//                may still read C_{j,j-1}.
//   FULL(i, c)   L_ic = (A_ic - sum_{k < c} L_ik L_ck^T) Linv_c^T   (i >= c + 2, and the right-hand side)
// Order: for j = 0, 1, ...: DIAGP(j), SUBP(j), CRIT(j), FULL(j+2 .. nb-1, j), FULL(nb, j). Every task
// waits only on tasks with smaller tickets, which were claimed by running workgroups (the chain
// workgroup's rule is given in the kernel), so the waits always end whatever the number of
// resident workgroups. Only CRIT steps lie on the critical path: the accumulations run ahead on
// the other workgroups.
//
// Hand-over: a producer's stores complete (s_waitcnt), then one thread writes back its L2, waits
// for the write-back and stores the tile's flag (the solve's epoch); a consumer polls the flag with
// agent-scope loads, invalidates its caches and waits for the invalidation before any wavefront
// reads the tile (release_flag / acquire_done). A wait that outlasts its deadline aborts the whole
// solve (all workgroups drain, the step is marked failed and reported).
enum { TASK_CRIT = 0, TASK_DIAGP = 1, TASK_SUBP = 2, TASK_FULL = 3 };

struct CholSync {
  int* bflag;   // [nb] (unused: the substitutions exchange tagged entries, see wait_tagged)
  int* fin;     // [(nb + 1) * nb] final L tile (i, c) at fin[i * nb + c]
  int* pdiag;   // [nb] partial diagonal tile of DIAGP(j)
  int* psub;    // [nb] partial sub-diagonal tile of SUBP(j)
  int* dinv;    // [nb] Linv_j published
  int* ctr;     // [1] ticket counter (0 between solves)
  int* abort_;  // [1] epoch of an aborted solve
  int* fflag;   // [nb] (unused, as bflag)
};

__host__ __device__ inline CholSync chol_sync(int* base, int nb) {
  CholSync S;
  S.bflag = base;
  S.fin = S.bflag + nb;
  S.pdiag = S.fin + (size_t)(nb + 1) * nb;
  S.psub = S.pdiag + nb;
  S.dinv = S.psub + nb;
  S.ctr = S.dinv + nb;
  S.abort_ = S.ctr + 1;
  S.fflag = S.abort_ + 1;
  return S;
}

// Task groups: group j holds DIAGP(j), SUBP(j) (from j = 2), CRIT(j), FULL(j + 2 .. nb - 1, j) and
// FULL(nb, j), in that ticket order; it has
//   g(j) = (j >= 2 ? 2 : 0) + 1 + max(nb - j - 2, 0) + 1
// tasks. group_start(j) = g(0) + ... + g(j - 1) in closed form: g(0) = 2 + max(nb - 2, 0),
// g(1) = 2 + max(nb - 3, 0), g(q) = nb + 2 - q for 2 <= q <= nb - 2 and g(nb - 1) = 4 (nb >= 3).
__host__ __device__ inline int group_start(int j, int nb) {
  if (j <= 0) return 0;
  const int g0 = 2 + (nb - 2 > 0 ? nb - 2 : 0);
  if (j == 1) return g0;
  const int g1 = 2 + (nb - 3 > 0 ? nb - 3 : 0);
  const int m = (j < nb - 1) ? j : nb - 1;  // groups 2 .. m - 1 have nb + 2 - q tasks
  int t = g0 + g1;
  if (m > 2) t += (m - 2) * (nb + 2) - ((m - 1) * m / 2 - 1);
  if (j >= nb && nb - 1 >= 2) t += 4;  // the last group
  return t;
}

__host__ __device__ inline int chol_task_count(int nb) { return group_start(nb, nb); }

__device__ __forceinline__ void decode_task(int t, int nb, int& kind, int& i, int& c) {
  if (t < 0 || t >= group_start(nb, nb)) {
    kind = -1;
    i = c = 0;
    return;
  }
  int lo = 0, hi = nb - 1;  // the group j with group_start(j) <= t < group_start(j + 1)
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (group_start(mid, nb) <= t) lo = mid;
    else hi = mid - 1;
  }
  const int j = lo;
  const int nfull = (nb - j - 2 > 0 ? nb - j - 2 : 0) + 1;
  int r = t - group_start(j, nb);
  if (j >= 2) {
    if (r == 0) { kind = TASK_DIAGP; i = j; c = j; return; }
    if (r == 1) { kind = TASK_SUBP; i = j; c = j - 1; return; }
    r -= 2;
  }
  if (r == 0) { kind = TASK_CRIT; i = j; c = j; return; }
  r -= 1;
  kind = TASK_FULL;
  i = (r < nfull - 1) ? j + 2 + r : nb;
  c = j;
}

__device__ __forceinline__ int ld_flag(const int* f) {
  return __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A wait that gives up (its deadline passed, or another wait of the solve gave up) marks the solve
// failed: the abort word stops every other wait of the solve, and the step is rejected and
// reported (TT_DEVERR_CHOL_SYNC), whichever task gave up and whether or not any ticket is left to
// claim.
__device__ __forceinline__ void mark_failed(const CholSync& S, LMScalars* sc, int epoch) {
  __hip_atomic_store(S.abort_, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  sc->chol_fail = 1;
  sc->err = TT_DEVERR_CHOL_SYNC;
}

// Thread 0 waits until every non-null flag equals epoch (the flags are read together, one round
// trip per poll), then acquires; the block learns the result. The wait gives up wait_ticks
// (constant-clock ticks) after it began.
__device__ bool block_wait(const int* f0, const int* f1, const int* f2, int epoch, const CholSync& S,
                           LMScalars* sc, uint64_t wait_ticks, int* s_ok) {
  if (threadIdx.x == 0) {
    const uint64_t deadline = __builtin_amdgcn_s_memrealtime() + wait_ticks;
    bool ok = true;
    const int* g0 = f0 ? f0 : S.abort_;
    const int* g1 = f1 ? f1 : S.abort_;
    const int* g2 = f2 ? f2 : S.abort_;
    int spins = 0;
    for (;;) {
      const int v0 = ld_flag(g0), v1 = ld_flag(g1), v2 = ld_flag(g2);
      if ((!f0 || v0 == epoch) && (!f1 || v1 == epoch) && (!f2 || v2 == epoch)) break;
      if ((++spins & 15) == 0 && (ld_flag(S.abort_) == epoch || __builtin_amdgcn_s_memrealtime() > deadline)) {
        ok = false;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    if (!ok) mark_failed(S, sc, epoch);
    acquire_done();
    *s_ok = ok ? 1 : 0;
  }
  __syncthreads();
  return *s_ok != 0;
}

// Wavefront 0 finds how many consecutive k >= k0 (< nk) have both tiles fi[k] and fc[k] final,
// waiting until at least one has; then acquires. Returns 0 if the solve was aborted.
__device__ int block_ready_prefix(const int* fi, const int* fc, int k0, int nk, int epoch, const CholSync& S,
                                  LMScalars* sc, uint64_t wait_ticks, int* s_val) {
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    const uint64_t deadline = __builtin_amdgcn_s_memrealtime() + wait_ticks;
    int pre = 0, spins = 0;
    for (;;) {
      const int k = k0 + lane;
      const bool r = (k >= nk) || (ld_flag(fi + k) == epoch && ld_flag(fc + k) == epoch);
      const unsigned long long m = __ballot(r);
      pre = (~m == 0ull) ? 64 : __builtin_ctzll(~m);
      if (pre > nk - k0) pre = nk - k0;
      if (pre > 0) break;
      if ((++spins & 15) == 0 &&
          (ld_flag(S.abort_) == epoch || __builtin_amdgcn_s_memrealtime() > deadline)) {
        if (lane == 0) mark_failed(S, sc, epoch);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    if (lane == 0) {
      acquire_done();
      *s_val = pre;
    }
  }
  __syncthreads();
  return *s_val;
}

// Operand tiles of one column k of a tile task in registers: rows of block i and of block c.
struct Stage32 {
  float4 v[4];
};
struct Stage16 {
  u32x4 v[2];
};

// acc += sum over the finished columns k < nk of the tile task's products, in column order. The
// operand tiles of the next two columns are in flight (two register stages, column k in stage
// k mod 2) while the product of column k runs, so a column's loads are issued two products before
// it is needed. A column is loaded only once both its tiles are known to be final (flags seen,
// then acquired); one that is not yet known is waited for after the product before it. load(k,
// a, b) issues column k's tiles into a stage, to_lds(a, b) moves a stage into the operand tiles
// in LDS, mma() runs the product. Returns false if the solve was aborted while waiting.
template <class T, class Load, class ToLds, class Mma>
__device__ __forceinline__ bool accumulate_columns(int nk, const int* fi, const int* fc, int epoch, const CholSync& S,
                                                   LMScalars* sc, uint64_t wt, int* s_val, Load load, ToLds to_lds,
                                                   Mma mma) {
  int kr = block_ready_prefix(fi, fc, 0, nk, epoch, S, sc, wt, s_val);  // columns < kr are known final
  if (kr == 0) return false;
  T a0, b0, a1, b1;
  load(0, a0, b0);
  int issued = 1;  // columns < issued are loaded or in flight
  if (nk > 1 && kr > 1) {
    load(1, a1, b1);
    issued = 2;
  }
  // issued, kr and nk are the same in every thread, so every barrier below is reached by all
  auto step = [&](int k, T& ca, T& cb, T& oa, T& ob) -> bool {
    __syncthreads();
    to_lds(ca, cb);
    __syncthreads();
    if (issued == k + 1 && k + 1 < nk && k + 1 < kr) {
      load(k + 1, oa, ob);
      issued = k + 2;
    }
    if (issued == k + 2 && k + 2 < nk && k + 2 < kr) {
      load(k + 2, ca, cb);
      issued = k + 3;
    }
    mma();
    if (issued == k + 1 && k + 1 < nk) {
      const int more = block_ready_prefix(fi, fc, k + 1, nk, epoch, S, sc, wt, s_val);
      if (more == 0) return false;
      kr = k + 1 + more;
      load(k + 1, oa, ob);
      issued = k + 2;
      if (k + 2 < nk && k + 2 < kr) {
        load(k + 2, ca, cb);
        issued = k + 3;
      }
    }
    return true;
  };
  for (int k = 0; k < nk; k += 2) {
    if (!step(k, a0, b0, a1, b1)) return false;
    if (k + 1 < nk && !step(k + 1, a1, b1, a0, b0)) return false;
  }
  return true;
}

// All stores of the block complete, then thread 0 raises the flag.
__device__ __forceinline__ void block_publish(int* f, int epoch) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) publish_flag(f, epoch);
}

// acc += X Y^T for 64 x 64 tiles X, Y in LDS (leading dimension LDS_LD). Four wavefronts each
// own a 32 x 32 quadrant as 2 x 2 MFMA 16x16x4 accumulators; acc[a][b][r] holds element
// (qr + 16 a + 4 (lane / 16) + r, qc + 16 b + lane % 16) with (qr, qc) = 32 (w / 2, w % 2).
__device__ __forceinline__ void mma64_acc(const float (*X)[LDS_LD], const float (*Y)[LDS_LD], floatx4 acc[2][2]) {
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  const int qr = 32 * (w / 2), qc = 32 * (w % 2);
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

// Row / column of element r of accumulator (a, b) of this thread (quadrant layout).
__device__ __forceinline__ int acc_row(int a, int r) {
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  return 32 * (w / 2) + 16 * a + 4 * (lane / 16) + r;
}
__device__ __forceinline__ int acc_col(int b) {
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  return 32 * (w % 2) + 16 * b + lane % 16;
}

// 64 x 64 tile at (r0, c0) of a row-major matrix into registers, 4 float4 per thread.
__device__ __forceinline__ void tile_load(const float* __restrict__ M, int ld, size_t r0, size_t c0, float4 v[4]) {
#pragma unroll
  for (int q = 0; q < 4; q++) {
    const int e = threadIdx.x + 256 * q;
    v[q] = *reinterpret_cast<const float4*>(M + (r0 + (e >> 4)) * ld + c0 + 4 * (e & 15));
  }
}
__device__ __forceinline__ void tile_to_lds(float (*X)[LDS_LD], const float4 v[4]) {
#pragma unroll
  for (int q = 0; q < 4; q++) {
    const int e = threadIdx.x + 256 * q;
    const int r = e >> 4, c = 4 * (e & 15);
    X[r][c] = v[q].x;
    X[r][c + 1] = v[q].y;
    X[r][c + 2] = v[q].z;
    X[r][c + 3] = v[q].w;
  }
}

// Tile (r0, c0) in the accumulator layout, equilibrated by dscale when scale is set.
__device__ __forceinline__ void acc_load(const float* __restrict__ A, int ld, size_t r0, size_t c0,
                                         const float* __restrict__ dscale, bool scale, floatx4 v[2][2]) {
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int b = 0; b < 2; b++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const size_t row = r0 + acc_row(a, r), col = c0 + acc_col(b);
        const float s0 = scale ? dscale[row] * dscale[col] : 1.0f;
        v[a][b][r] = A[row * ld + col] * s0;
      }
}
__device__ __forceinline__ void acc_store(float* __restrict__ A, int ld, size_t r0, size_t c0, const floatx4 v[2][2]) {
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int b = 0; b < 2; b++)
#pragma unroll
      for (int r = 0; r < 4; r++) st_coh(&A[(r0 + acc_row(a, r)) * ld + c0 + acc_col(b)], v[a][b][r]);
}
__device__ __forceinline__ void acc_to_lds(float (*X)[LDS_LD], const floatx4 v[2][2], bool lower_only) {
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int b = 0; b < 2; b++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int row = acc_row(a, r), col = acc_col(b);
        X[row][col] = (!lower_only || col <= row) ? v[a][b][r] : 0.0f;
      }
}
__device__ __forceinline__ void acc_zero(floatx4 v[2][2]) {
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int b = 0; b < 2; b++) v[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
}

// ---- 16-bit tile products (precision forms) --------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
constexpr int LD16 = NB + 8;  // 16-bit LDS tiles: rows of 144 bytes (16-byte aligned)

// FP32 -> bfloat16 bits, round to nearest even (finite inputs) / FP32 -> binary16 bits.
__device__ __forceinline__ uint16_t to_bf16(float f) {
  const uint32_t u = __float_as_uint(f);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ uint16_t to_f16(float f) {
  const _Float16 h = (_Float16)f;
  return __builtin_bit_cast(uint16_t, h);
}

// 16-bit copy of a tile held in the accumulator layout.
__device__ __forceinline__ void acc_store16(uint16_t* __restrict__ A16, int ld, size_t r0, size_t c0,
                                            const floatx4 v[2][2], int prec) {
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int b = 0; b < 2; b++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const float f = v[a][b][r];
        st_coh16(&A16[(r0 + acc_row(a, r)) * ld + c0 + acc_col(b)], (prec == TT_BF16_IR) ? to_bf16(f) : to_f16(f));
      }
}

// 64 x 64 16-bit tile at (r0, c0) into registers (two 16-byte pieces per thread) and into LDS.
__device__ __forceinline__ void tile_load16(const uint16_t* __restrict__ M, int ld, size_t r0, size_t c0, u32x4 v[2]) {
#pragma unroll
  for (int q = 0; q < 2; q++) {
    const int e = threadIdx.x + 256 * q;  // 512 pieces of 8 elements: row e / 8, columns 8 (e % 8)
    v[q] = *reinterpret_cast<const u32x4*>(M + (r0 + (e >> 3)) * ld + c0 + 8 * (e & 7));
  }
}
__device__ __forceinline__ void tile16_to_lds(uint16_t* X, const u32x4 v[2]) {
#pragma unroll
  for (int q = 0; q < 2; q++) {
    const int e = threadIdx.x + 256 * q;
    *reinterpret_cast<u32x4*>(X + (e >> 3) * LD16 + 8 * (e & 7)) = v[q];
  }
}

// acc += X Y^T for 64 x 64 16-bit tiles in LDS (v_mfma_f32_16x16x32_{bf16,f16}, FP32 accumulation),
// same quadrant layout as mma64_acc. Lane (li, lk) supplies the 8 consecutive reduction indices
// 32 s + 8 lk .. + 7 of step s for both operands, so the two 32-step halves cover all 64.
__device__ __forceinline__ void mma64_acc16(const uint16_t* X, const uint16_t* Y, floatx4 acc[2][2], int prec) {
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  const int qr = 32 * (w / 2), qc = 32 * (w % 2);
  const int li = lane % 16, k8 = 8 * (lane / 16);
#pragma unroll
  for (int s = 0; s < 2; s++) {
    u32x4 av[2], bv[2];
#pragma unroll
    for (int a = 0; a < 2; a++) av[a] = *reinterpret_cast<const u32x4*>(X + (qr + 16 * a + li) * LD16 + 32 * s + k8);
#pragma unroll
    for (int b = 0; b < 2; b++) bv[b] = *reinterpret_cast<const u32x4*>(Y + (qc + 16 * b + li) * LD16 + 32 * s + k8);
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
      for (int b = 0; b < 2; b++) {
        if (prec == TT_BF16_IR)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av[a]),
                                                               __builtin_bit_cast(bf16x8, bv[b]), acc[a][b], 0, 0, 0);
        else
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(halfx8, av[a]),
                                                              __builtin_bit_cast(halfx8, bv[b]), acc[a][b], 0, 0, 0);
      }
  }
}

struct CholArgs {
  float* A;
  int ld, npad, nb, ntasks;
  int which;         // substitutions: index of the launch within the solve (tags its entries)
  const float* dscale;
  float* Linv;
  int* flags;
  LMScalars* sc;
  float* x;          // solution of the back substitution
  int prec;          // TT_FP32, TT_BF16_IR or TT_FP16_IR: input type of the tile products
  uint16_t* A16;     // 16-bit copies of the finished L tiles (same layout as A), or null
  const float* A0;   // refinement: the damped matrix before factorisation (lower triangle), or null
  const float* c;    // refinement: the equilibrated right-hand side
  double* xd;        // refinement: the solution accumulated in FP64 [npad], then the residual's
                     // partial sums [nb][nb][64]
  uint64_t* tw;      // [npad] tagged solution entries exchanged inside a substitution
};

// Ticket of CRIT(j): the number of tasks in the groups before j, plus DIAGP(j) and SUBP(j).
__device__ __forceinline__ int crit_ticket(int j, int nb) { return group_start(j, nb) + (j >= 2 ? 2 : 0); }

enum { MODE_TASK = 0, MODE_CRIT = 1, MODE_RETRY = 2 };

// C_{j,j-1} (j >= 1) in tile layout: for j = 1 the raw block A_{1,0}, equilibrated here (only the
// chain reads it: its own step 1 overwrites the tile with L_{1,0}); later SUBP(j)'s partial tile,
// kept in the upper-triangle tile (j-1, j).
__device__ __forceinline__ void csub_load(const CholArgs& P, int j, float4 va[4]) {
  const size_t rj = (size_t)NB * j;
  if (j >= 2) {
    tile_load(P.A, P.ld, rj - NB, rj, va);
    return;
  }
  tile_load(P.A, P.ld, rj, rj - NB, va);
  {
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int e = threadIdx.x + 256 * q;
      const float sr = P.dscale[NB + (e >> 4)];
      const int cc = 4 * (e & 15);
      va[q].x *= sr * P.dscale[cc];
      va[q].y *= sr * P.dscale[cc + 1];
      va[q].z *= sr * P.dscale[cc + 2];
      va[q].w *= sr * P.dscale[cc + 3];
    }
  }
}

// The chain's inputs for step j: C_{j,j-1} (tile layout) and C_jj (accumulator layout). For j <= 1
// these are the raw, not yet equilibrated blocks of A; later they are the partial tiles, loaded as
// they are (no arithmetic on the loaded values, so that a prefetch leaves them in flight until the
// step uses them).
__device__ __forceinline__ void chain_load(const CholArgs& P, int j, float4 va[4], floatx4 cp[2][2]) {
  const size_t rj = (size_t)NB * j;
  if (j >= 2) {
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
      for (int b = 0; b < 2; b++)
#pragma unroll
        for (int r = 0; r < 4; r++) cp[a][b][r] = P.A[(rj + acc_row(a, r)) * P.ld + rj + acc_col(b)];
    tile_load(P.A, P.ld, rj - NB, rj, va);
    return;
  }
  acc_load(P.A, P.ld, rj, rj, P.dscale, true, cp);
  if (j >= 1) csub_load(P, j, va);
}

// Up to kMaxCholBatch independent systems per launch, passed by value (no upload per solve).
constexpr int kMaxCholBatch = 32;
struct CholBatch {
  int nprob;
  uint64_t wait_ticks;  // how long one hand-over wait may last, in constant-clock ticks
  CholArgs p[kMaxCholBatch];
};

enum { MODE_EXIT = 3 };

// What thread 0 needs of a system to claim its tasks, kept in registers (reading the kernel
// arguments with a per-thread index costs a memory round trip).
struct SysRef {
  int* ctr;
  const int* abort_;
  int ntasks, epoch, nb;
};
__device__ __forceinline__ SysRef sys_ref(const CholBatch& B, int q) {
  const CholArgs& Q = B.p[q];
  const CholSync S = chol_sync(Q.flags, Q.nb);
  // the solve's epoch, set by the damping kernel that ran before this launch
  const int epoch = __hip_atomic_load(&Q.sc->solve_epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return SysRef{S.ctr, S.abort_, Q.ntasks, epoch, Q.nb};
}

__global__ __launch_bounds__(256) void k_chol_dataflow(const CholBatch B) {
  __shared__ __attribute__((aligned(16))) float X[NB][LDS_LD];
  __shared__ __attribute__((aligned(16))) float Y[NB][LDS_LD];
  __shared__ __attribute__((aligned(16))) float Z[NB][LDS_LD];  // the chain's Linv_{j-1} between CRIT steps
  static_assert(POTRF_SCRATCH_FLOATS <= NB * LDS_LD, "factorisation scratch must fit in one tile buffer");
  __shared__ int s_task, s_val, s_val2, s_mode, s_prob, s_ctr, s_pubcnt, s_fast, s_ep;
  const int tid = threadIdx.x;
  const uint64_t wt = B.wait_ticks;
  if (tid == 0) s_pubcnt = 0;
  // the six tiles above the diagonal of the chain's inverse stay zero: the factorisation writes only
  // the lower ones, and nothing else writes Z (the first barrier of the loop orders this)
  for (int e = tid; e < 6 * 256; e += 256) {
    const int t = e >> 8, w = e & 255;
    const int r = (t < 3) ? 0 : (t < 5 ? 1 : 2);
    const int c = (t < 3) ? 1 + t : (t < 5 ? t - 1 : 3);
    Z[16 * r + (w >> 4)][16 * c + (w & 15)] = 0.0f;
  }
  // Each system has its own ticket counter and task order. A workgroup visits the systems in a
  // cyclic order starting at blockIdx % nprob, claiming tasks from one until its counter runs out
  // (one failing claim per system per workgroup, so the claim that returns ntasks + gridDim - 1
  // is a system's last and rearms its counter for the next solve), then moves to the next.
  //
  // The workgroup that claims a system's ticket 0 (CRIT(0)) runs that system's whole critical
  // chain CRIT(0..nb-1) and keeps each Linv_j in LDS for the next step; CRIT tickets claimed by
  // others are empty. Before CRIT(j) may wait on DIAGP(j) and SUBP(j), their tickets must have
  // been handed out: until the counter has passed them, the chain workgroup claims the system's
  // next ticket itself (compare-and-swap, so it never takes one at or beyond CRIT(j)) and runs
  // that task, which depends only on smaller tickets of the same system. Tasks of different systems
  // never wait on each other, so every wait ends whatever the number of resident workgroups.
  int cur = (int)blockIdx.x % B.nprob;  // thread 0: system being claimed from
  int vis = 0;                          // thread 0: systems whose counter this workgroup exhausted
  SysRef qc = {}, qh = {};              // thread 0: the chain's system and system cur
  if (tid == 0) qh = sys_ref(B, cur);
  int chain = -1, chain_p = 0;
  int ctr_seen = 0;          // thread 0: last counter value read by the chain (the counter only grows)
  bool have_pref = false;    // the chain's inputs for its next step are already in cva / ccp
  float4 cva[4];             // chain prefetch: C_{j,j-1} (tile layout)
  floatx4 ccp[2][2];         // chain prefetch: C_jj (accumulator layout)
  for (;;) {
    __syncthreads();  // every thread is done with the shared scalars of the previous step
    if (tid == 0) {
      int t = -1, mode = MODE_TASK, prob = cur;
      bool chain_fast = false;
      if (chain >= 0) {
        // the chain's system fields are kept in registers: reading them from the kernel
        // arguments here, in code only thread 0 runs, would cost a memory round trip per step
        prob = chain_p;
        int* ctr = qc.ctr;
        const int need = crit_ticket(chain, qc.nb);
        if (ctr_seen < need) ctr_seen = max(ctr_seen, s_ctr);  // the look ahead's reading
        if (ctr_seen >= need) {
          mode = MODE_CRIT;
          chain_fast = true;
        } else {
          // Only this path waits for memory, and the wait stays inside it (the previous step's
          // flag store may still be in flight, and a wait here would wait for it too).
          const int c0 = ld_flag(ctr);
          ctr_seen = c0;
          if (c0 >= need) {
            mode = MODE_CRIT;
            chain_fast = true;
          } else {
            int expect = c0;
            mode = __hip_atomic_compare_exchange_strong(ctr, &expect, c0 + 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT)
                       ? MODE_TASK
                       : MODE_RETRY;
            t = c0;
          }
        }
      } else if (vis >= B.nprob) {
        mode = MODE_EXIT;
      } else {
        // the abort word is read in the same round trip as the claim
        const int ab = ld_flag(qh.abort_);
        t = __hip_atomic_fetch_add(qh.ctr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (t >= qh.ntasks) {
          if (t == qh.ntasks + (int)gridDim.x - 1) __hip_atomic_store(qh.ctr, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          vis++;
          cur = (cur + 1 == B.nprob) ? 0 : cur + 1;
          if (vis < B.nprob) qh = sys_ref(B, cur);
          mode = MODE_RETRY;
        }
        s_val = (mode == MODE_TASK) && (ab == qh.epoch);
      }
      s_task = t;
      s_mode = mode;
      s_prob = prob;
      s_ep = (chain >= 0) ? qc.epoch : qh.epoch;  // the claimed task's system (MODE_TASK, MODE_CRIT)
      // the chain's waits watch the abort word themselves; a task the chain claims checks it here
      if (chain >= 0) s_val = (chain_fast || mode != MODE_TASK) ? 0 : (ld_flag(qc.abort_) == qc.epoch);
    }
    __syncthreads();
    const int t = s_task, mode = s_mode, prob = s_prob;
    const bool aborted = s_val != 0;
    if (mode == MODE_EXIT) break;
    if (mode == MODE_RETRY) continue;
    const CholArgs& P = B.p[prob];
    const int nb = P.nb, ld = P.ld, epoch = s_ep;
    const CholSync S = chol_sync(P.flags, nb);
    if (aborted) {
      if (tid == 0) {
        P.sc->chol_fail = 1;
        P.sc->err = TT_DEVERR_CHOL_SYNC;
      }
      if (mode == MODE_CRIT) chain = -1;
      continue;
    }
    floatx4 acc[2][2], cpre[2][2];
    if (mode == MODE_CRIT) {
      // Consecutive chain steps run back to back without the claim at the top of the loop while
      // the next step's partial tiles are already loaded and the ticket counter (as last read)
      // has passed its CRIT ticket, i.e. while the claim would only confirm the chain's turn.
      for (int j = chain;;) {
        const size_t rj = (size_t)NB * j;
        chain = (j + 1 < nb) ? j + 1 : -1;
        if (!have_pref) {
          if (j >= 2 && !block_wait(S.pdiag + j, S.psub + j, nullptr, epoch, S, P.sc, wt, &s_val)) {
            chain = -1;
            break;
          }
          chain_load(P, j, cva, ccp);
        }
        have_pref = false;
        acc_to_lds(Y, ccp, true);
        if (j >= 1) tile_to_lds(X, cva);
        __syncthreads();
        if (j >= 1) {
          // L_{j,j-1} = C_{j,j-1} Linv_{j-1}^T: wavefront g computes rows 16 g .. 16 g + 15 (four
          // 16 x 16 tiles), then overwrites those rows of X (wavefronts 1-3 store the whole tile
          // during the factorisation's first phase). Linv is lower triangular, so column block c
          // only sums over the blocks k0 <= 16 c.
          const int g = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
          floatx4 t4[4];
  #pragma unroll
          for (int c = 0; c < 4; c++) {
            t4[c] = mm16_abt<LDS_LD, LDS_LD>(&X[16 * g][0], &Z[16 * c][0], floatx4{0.f, 0.f, 0.f, 0.f}, c + 1);
          }
  #pragma unroll
          for (int c = 0; c < 4; c++)
  #pragma unroll
            for (int q = 0; q < 4; q++) {
              X[16 * g + 4 * lk + q][16 * c + li] = t4[c][q];
            }
          __syncthreads();
        }
        // Z = Linv_j, kept for step j + 1; for j >= 1 the update C_jj -= L_{j,j-1} L_{j,j-1}^T is folded
        // into the factorisation's first phase, which also publishes L_{j,j-1}
        // the look ahead: the next step's partial tiles (from step 2 on) and the ticket counter
        ChainPoll poll;
        poll.f0 = (j + 1 >= 2 && j + 1 < nb) ? S.pdiag + j + 1 : nullptr;
        poll.f1 = (j + 1 >= 2 && j + 1 < nb) ? S.psub + j + 1 : nullptr;
        poll.ctr = S.ctr;
        poll.epoch = epoch;
        poll.s_ready = &s_val;
        poll.s_ctr = &s_ctr;
        poll.s_ready2 = &s_val2;
        // wavefronts 1-3: L_{j,j-1} (X) to tile (j, j-1) of A and of its 16-bit copy
        // (every LDS read is issued before the first store, and the pointers are locals: the stores'
        // memory clobber would otherwise order each read after the previous store)
        auto ustore = [&]() {
          const size_t o0 = rj * ld + rj - NB;
          float* const A = P.A + o0;
          const int prec = P.prec;
          uint16_t* const A16 = (prec != TT_FP32) ? P.A16 + o0 : nullptr;
          const int e0 = tid - 64;
          float4 v[6];
#pragma unroll
          for (int k = 0; k < 6; k++) {
            const int e = min(e0 + 192 * k, NB * NB / 4 - 1), row = e >> 4, c4 = 4 * (e & 15);
            const float2 lo = *reinterpret_cast<const float2*>(&X[row][c4]);
            const float2 hi = *reinterpret_cast<const float2*>(&X[row][c4 + 2]);
            v[k] = make_float4(lo.x, lo.y, hi.x, hi.y);
          }
#pragma unroll
          for (int k = 0; k < 6; k++) {
            const int e = e0 + 192 * k;
            if (e < NB * NB / 4) {
              const size_t o = (size_t)(e >> 4) * ld + 4 * (e & 15);
              st_coh4(A + o, v[k]);
              if (prec != TT_FP32) {
                const bool b = prec == TT_BF16_IR;
                const uint64_t h0 = b ? to_bf16(v[k].x) : to_f16(v[k].x), h1 = b ? to_bf16(v[k].y) : to_f16(v[k].y);
                const uint64_t h2 = b ? to_bf16(v[k].z) : to_f16(v[k].z), h3 = b ? to_bf16(v[k].w) : to_f16(v[k].w);
                st_coh16x4(A16 + o, h0 | (h1 << 16) | (h2 << 32) | (h3 << 48));
              }
            }
          }
        };
        // once the look ahead (fourth phase) has found the next step's partial tiles published, their
        // loads are issued at once and overlap the last phase and the stores of Linv_j
        bool early = false;
        auto pre = [&]() {
          if (j + 1 >= 2 && j + 1 < nb && s_val) {
            chain_load(P, j + 1, cva, ccp);
            early = true;
          }
        };
        const bool ok = (j >= 1) ? potrf_trtri64(Y, Z, &X[0][0], X, S.fin + (size_t)j * nb + (j - 1), epoch, &poll,
                                                 &s_pubcnt, ustore, pre)
                                 : potrf_trtri64(Y, Z, &X[0][0], nullptr, nullptr, 0, &poll, nullptr, NoOp(), pre);
        // the second look (fifth phase) found them: their loads overlap the stores of Linv_j
        if (!early && j + 1 >= 2 && j + 1 < nb && s_val2) {
          chain_load(P, j + 1, cva, ccp);
          early = true;
        }
        {
          float* const Lj = P.Linv + (size_t)j * NB * NB;
          float4 v[4];
#pragma unroll
          for (int k = 0; k < 4; k++) {
            const int e = tid + 256 * k, r = e >> 4, cc = 4 * (e & 15);
            const float2 lo = *reinterpret_cast<const float2*>(&Z[r][cc]);
            const float2 hi = *reinterpret_cast<const float2*>(&Z[r][cc + 2]);
            v[k] = make_float4(lo.x, lo.y, hi.x, hi.y);
          }
#pragma unroll
          for (int k = 0; k < 4; k++) {
            const int e = tid + 256 * k;
            st_coh4(Lj + (e >> 4) * NB + 4 * (e & 15), v[k]);
          }
        }
        if (tid == 0 && !ok) P.sc->chol_fail = 1;
        // If the look ahead did not find the next step's partial tiles ready, look once more; if they
        // are, their loads overlap the completion of the Linv_j stores that the publication below
        // waits for.
        if (j + 1 < nb) {
          bool ready = early;
          if (!ready) {
            __syncthreads();  // every thread has read s_val
            if (tid == 0) {
              const int v0 = ld_flag(S.pdiag + j + 1), v1 = ld_flag(S.psub + j + 1);
              const bool r = (v0 == epoch) && (v1 == epoch);
              if (r) acquire_done();
              s_val = r ? 1 : 0;
            }
            __syncthreads();
            ready = s_val != 0;
            if (ready) chain_load(P, j + 1, cva, ccp);
          }
          have_pref = ready;
        }
        if (tid == 0) {
          bool f = false;
          if (chain >= 0 && have_pref) {
            const int need = crit_ticket(chain, qc.nb);
            if (ctr_seen < need) ctr_seen = max(ctr_seen, s_ctr);
            f = ctr_seen >= need;
          }
          s_fast = f ? 1 : 0;
        }
        block_publish(S.dinv + j, epoch);  // its barrier also shares s_fast
        if (!s_fast) break;
        j = chain;
      }
      continue;
    }
    int kind, i, c;
    decode_task(t, nb, kind, i, c);
    if (kind == TASK_CRIT) {
      if (i == 0) {  // this workgroup runs the system's critical chain
        chain = 0;
        chain_p = prob;
        if (tid == 0) {
          qc = sys_ref(B, prob);
          ctr_seen = 0;
          s_ctr = 0;
        }
      }
      continue;
    }
    // DIAGP / SUBP / FULL: accumulate the finished columns k < nk into the tile (SUBP's last
    // column, k = c - 1, follows below)
    const int nk = (kind == TASK_FULL) ? c : c - 1;
    const size_t ri = (i < nb) ? (size_t)NB * i : (size_t)P.npad;
    const size_t rc = (size_t)NB * c;
    const bool same = (i == c);
    acc_load(P.A, ld, ri, rc, P.dscale, i < nb, cpre);
    acc_zero(acc);
    const int* fi = S.fin + (size_t)i * nb;
    const int* fc = S.fin + (size_t)c * nb;
    bool ok = true;
    if (nk > 0 && P.prec != TT_FP32) {
      // 16-bit operand tiles (half the bytes)
      uint16_t* X16 = reinterpret_cast<uint16_t*>(&X[0][0]);
      uint16_t* Y16 = reinterpret_cast<uint16_t*>(&Y[0][0]);
      ok = accumulate_columns<Stage16>(
          nk, fi, fc, epoch, S, P.sc, wt, &s_val,
          [&](int k, Stage16& a, Stage16& b) {
            tile_load16(P.A16, ld, ri, (size_t)NB * k, a.v);
            if (!same) tile_load16(P.A16, ld, rc, (size_t)NB * k, b.v);
          },
          [&](const Stage16& a, const Stage16& b) {
            tile16_to_lds(X16, a.v);
            if (!same) tile16_to_lds(Y16, b.v);
          },
          [&]() { mma64_acc16(X16, same ? X16 : Y16, acc, P.prec); });
    } else if (nk > 0) {
      ok = accumulate_columns<Stage32>(
          nk, fi, fc, epoch, S, P.sc, wt, &s_val,
          [&](int k, Stage32& a, Stage32& b) {
            tile_load(P.A, ld, ri, (size_t)NB * k, a.v);
            if (!same) tile_load(P.A, ld, rc, (size_t)NB * k, b.v);
          },
          [&](const Stage32& a, const Stage32& b) {
            tile_to_lds(X, a.v);
            if (!same) tile_to_lds(Y, b.v);
          },
          [&]() {
            if (same) mma64_acc(X, X, acc);
            else mma64_acc(X, Y, acc);
          });
    }
    if (!ok) continue;
    if (kind == TASK_SUBP) {
      // last column m = c - 1 = i - 2: acc += L_{i,m} V^T with V = L_{c,m}, once FULL(i, m) is final.
      // For c >= 2, V = C_{c,m} Linv_m^T is formed here from SUBP(c)'s tile and Linv_m. For c = 1
      // the raw A_{1,0} is not there to form it from once CRIT(1) has begun (it overwrites tile
      // (1, 0) with L_{1,0}), so V is that tile, read once CRIT(1) has published it.
      const int m = c - 1;
      floatx4 vt[2][2];
      if (c >= 2) {
        if (!block_wait(S.dinv + m, S.psub + c, nullptr, epoch, S, P.sc, wt, &s_val)) continue;
        {
          float4 va[4], vb[4];
          csub_load(P, c, va);
          tile_load(P.Linv + (size_t)m * NB * NB, NB, 0, 0, vb);
          __syncthreads();
          tile_to_lds(X, va);
          tile_to_lds(Y, vb);
        }
        __syncthreads();
        acc_zero(vt);
        mma64_acc(X, Y, vt);
      }
      if (!block_wait(fi + m, c == 1 ? fc + m : nullptr, nullptr, epoch, S, P.sc, wt, &s_val)) continue;
      {
        float4 va[4];
        tile_load(P.A, ld, ri, (size_t)NB * m, va);
        if (c >= 2) {
          acc_to_lds(Y, vt, false);
        } else {
          float4 vb[4];
          tile_load(P.A, ld, rc, (size_t)NB * m, vb);
          tile_to_lds(Y, vb);
        }
        tile_to_lds(X, va);
      }
      __syncthreads();
      mma64_acc(X, Y, acc);
    }
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
      for (int b = 0; b < 2; b++) cpre[a][b] -= acc[a][b];
    if (kind != TASK_FULL) {
      if (kind == TASK_DIAGP) acc_store(P.A, ld, ri, rc, cpre);
      else acc_store(P.A, ld, rc, ri, cpre);  // upper-triangle tile (i - 1, i)
      block_publish(kind == TASK_DIAGP ? S.pdiag + i : S.psub + i, epoch);
      continue;
    }
    if (!block_wait(S.dinv + c, nullptr, nullptr, epoch, S, P.sc, wt, &s_val)) continue;
    {
      float4 vb[4];
      tile_load(P.Linv + (size_t)c * NB * NB, NB, 0, 0, vb);
      acc_to_lds(X, cpre, false);
      tile_to_lds(Y, vb);
    }
    __syncthreads();
    acc_zero(acc);
    mma64_acc(X, Y, acc);
    acc_store(P.A, ld, ri, rc, acc);
    if (P.prec != TT_FP32) acc_store16(P.A16, ld, ri, rc, acc, P.prec);
    block_publish(S.fin + (size_t)i * nb + c, epoch);
  }
}

constexpr long long kSpinLimit = 1ll << 22;

// Tag of the entries one substitution launch exchanges: the solve's epoch (set on the device by
// the damping kernel) and the launch's index within the solve (0: the back substitution of the
// factored right-hand side; 1 + 2t, 2 + 2t: forward and back substitution of refinement step t).
// Different launches of one solve, and launches of the previous solve, never share a tag; the tag
// is never 0 (the value the entries are cleared to).
__device__ __forceinline__ uint32_t subst_tag(const LMScalars* sc, int which) {
  const int e = __hip_atomic_load(&sc->solve_epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return ((uint32_t)(e & 0x3FFFFFF) << 5) + (uint32_t)which + 1u;
}

// Hand-over between the workgroups of a substitution: each solution entry travels as one 64-bit
// word (epoch << 32 | float bits) written and read with agent-scope atomics, so a consumer lane
// polls the entry it needs and gets the value with the same read that tells it the value is there
// (one memory round trip per block step, no separate flag). A bounded spin marks the solve failed.
__device__ __forceinline__ float wait_tagged(const uint64_t* w, uint32_t tag, bool& ok) {
  long long spins = 0;
  uint64_t v;
  while (((v = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) >> 32) != tag) {
    if (++spins > kSpinLimit) {
      ok = false;
      break;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  return __uint_as_float((uint32_t)v);
}
__device__ __forceinline__ void put_tagged(uint64_t* w, float x, uint32_t tag) {
  __hip_atomic_store(w, ((uint64_t)tag << 32) | __float_as_uint(x), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

// Back substitution L^T x = y (y in the right-hand-side row): one wavefront per block row, for a
// batch of systems laid out one after another over the grid (workgroups wg0[q] .. wg0[q+1]-1 serve
// system q, block rows from the last). Block row j folds in x_k of every later block as it arrives.
struct BackBatch {
  int nprob;
  int wg0[kMaxCholBatch + 1];
  CholArgs p[kMaxCholBatch];
};

__global__ __launch_bounds__(64) void k_chol_backsolve(const BackBatch B) {
  __shared__ float xs[NB];
  __shared__ float rs[NB];
  int q = 0;
  while (q + 1 < B.nprob && (int)blockIdx.x >= B.wg0[q + 1]) q++;
  const CholArgs& P = B.p[q];
  const int nb = P.nb, ld = P.ld;
  const uint32_t tag = subst_tag(P.sc, P.which);
  const float* __restrict__ A = P.A;
  const int j = nb - 1 - ((int)blockIdx.x - B.wg0[q]);
  const int c = threadIdx.x;
  const float* yrow = A + (size_t)P.npad * ld;
  const float y = yrow[NB * j + c];
  const float* Li = P.Linv + (size_t)j * NB * NB;
  float lic[NB];
#pragma unroll
  for (int m = 0; m < NB; m++) lic[m] = Li[m * NB + c];
  // four partial sums (entries m = 4 i + t into acc[t]) keep the dependent chain after each wait
  // short; they are added in a fixed order
  float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  bool ok = true;
  for (int k = nb - 1; k > j; k--) {
    // the tile column is final (written by the factorisation): fetch it before waiting
    float col[NB];
#pragma unroll
    for (int m = 0; m < NB; m++) col[m] = A[(size_t)(NB * k + m) * ld + NB * j + c];
    xs[c] = wait_tagged(P.tw + NB * k + c, tag, ok);
    __syncthreads();
#pragma unroll
    for (int m = 0; m < NB; m++) acc[m & 3] += col[m] * xs[m];
    __syncthreads();
  }
  rs[c] = y - ((acc[0] + acc[1]) + (acc[2] + acc[3]));
  __syncthreads();
  float sp[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int m = 0; m < NB; m++) sp[m & 3] += lic[m] * rs[m];
  const float s = (sp[0] + sp[1]) + (sp[2] + sp[3]);
  P.x[NB * j + c] = s;
  put_tagged(P.tw + NB * j + c, s, tag);
  if (!ok) {
    P.sc->chol_fail = 1;
    P.sc->err = TT_DEVERR_CHOL_SYNC;
  }
}

// Forward substitution y = L^{-1} r for the refinement steps (the first right-hand side rides
// along the factorisation): r is in the right-hand-side row and is overwritten by y. One wavefront
// per block row, in increasing order; block row j folds in y_k of every k < j as it arrives.
__global__ __launch_bounds__(64) void k_chol_fwdsolve(const BackBatch B) {
  __shared__ float ys[NB];
  __shared__ float rs[NB];
  int q = 0;
  while (q + 1 < B.nprob && (int)blockIdx.x >= B.wg0[q + 1]) q++;
  const CholArgs& P = B.p[q];
  const int ld = P.ld;
  const uint32_t tag = subst_tag(P.sc, P.which);
  float* row = P.A + (size_t)P.npad * ld;
  const int j = (int)blockIdx.x - B.wg0[q];
  const int c = threadIdx.x;
  const float rj = row[NB * j + c];
  // row c of Linv_jj, read before any wait (it is final when the launch starts), so that the last
  // block step after the wait reads only registers and LDS
  const float* Li = P.Linv + (size_t)j * NB * NB + (size_t)c * NB;
  float lir[NB];
#pragma unroll
  for (int m = 0; m < NB; m++) lir[m] = Li[m];
  float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};  // partial sums as in the back substitution
  bool ok = true;
  for (int k = 0; k < j; k++) {
    // row c of L_jk is final (written by the factorisation): fetch it before waiting
    const float4* Lr = reinterpret_cast<const float4*>(P.A + (size_t)(NB * j + c) * ld + NB * k);
    float4 lr[NB / 4];
#pragma unroll
    for (int m = 0; m < NB / 4; m++) lr[m] = Lr[m];
    ys[c] = wait_tagged(P.tw + NB * k + c, tag, ok);
    __syncthreads();
#pragma unroll
    for (int m = 0; m < NB / 4; m++) {
      acc[0] += lr[m].x * ys[4 * m];
      acc[1] += lr[m].y * ys[4 * m + 1];
      acc[2] += lr[m].z * ys[4 * m + 2];
      acc[3] += lr[m].w * ys[4 * m + 3];
    }
    __syncthreads();
  }
  rs[c] = rj - ((acc[0] + acc[1]) + (acc[2] + acc[3]));
  __syncthreads();
  float yp[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int m = 0; m < NB; m++) yp[m & 3] += lir[m] * rs[m];
  const float y = (yp[0] + yp[1]) + (yp[2] + yp[3]);
  row[NB * j + c] = y;  // read by the back substitution, a later launch
  put_tagged(P.tw + NB * j + c, y, tag);
  if (!ok) {
    P.sc->chol_fail = 1;
    P.sc->err = TT_DEVERR_CHOL_SYNC;
  }
}

// Refinement residual of the equilibrated system, r = c - D A0 D xd, formed in FP64 from the FP32
// damped matrix A0 (lower triangle) and the FP64 solution, in two launches. k_ir_resid_tiles: one
// workgroup per lower-triangle tile (i, k), k <= i, which it reads once: its row sums against
// (D xd) of block k are the part of block row i from block column k, and for k < i its column sums
// against (D xd) of block i are the part of block row k from block column i (the diagonal tile
// mirrors its lower triangle). Each part is stored in FP64 after the solution, at
// xd[npad + (row block * nb + column block) * 64 + row]. k_ir_resid_sum: block row i adds its nb
// parts in column order (the same order on every run) and writes r, rounded to FP32, into the
// right-hand-side row.
__device__ __forceinline__ int lower_tile_system(const BackBatch& B, int& t) {
  int q = 0;
  for (;;) {
    const int nb = B.p[q].nb, nt = nb * (nb + 1) / 2;
    if (t < nt || q + 1 >= B.nprob) return q;
    t -= nt;
    q++;
  }
}
__device__ __forceinline__ void lower_tile_of(int t, int& i, int& k) {  // t = i (i + 1) / 2 + k, k <= i
  i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= t) i++;
  while (i * (i + 1) / 2 > t) i--;
  k = t - i * (i + 1) / 2;
}

__global__ __launch_bounds__(256) void k_ir_resid_tiles(const BackBatch B) {
  __shared__ float T[NB][NB + 1];
  __shared__ double xr[NB], xc[NB];
  int t = (int)blockIdx.x;
  const CholArgs& P = B.p[lower_tile_system(B, t)];
  const int ld = P.ld, nb = P.nb, tid = threadIdx.x;
  int i, k;
  lower_tile_of(t, i, k);
#pragma unroll
  for (int u = 0; u < 4; u++) {
    const int e = tid + 256 * u, r = e >> 4, c = 4 * (e & 15);
    const float4 v = *reinterpret_cast<const float4*>(P.A0 + (size_t)(NB * i + r) * ld + NB * k + c);
    T[r][c] = v.x;
    T[r][c + 1] = v.y;
    T[r][c + 2] = v.z;
    T[r][c + 3] = v.w;
  }
  if (tid < NB) xc[tid] = (double)P.dscale[NB * k + tid] * P.xd[NB * k + tid];
  else if (tid < 2 * NB) xr[tid - NB] = (double)P.dscale[NB * i + tid - NB] * P.xd[NB * i + tid - NB];
  __syncthreads();
  double* part = P.xd + P.npad;
  if (tid < NB) {
    const int r = tid;
    double acc = 0.0;
    for (int c = 0; c < NB; c++) acc += (double)((i != k || c <= r) ? T[r][c] : T[c][r]) * xc[c];
    part[((size_t)i * nb + k) * NB + r] = acc;
  } else if (tid < 2 * NB && i != k) {
    const int c = tid - NB;
    double acc = 0.0;
    for (int r = 0; r < NB; r++) acc += (double)T[r][c] * xr[r];
    part[((size_t)k * nb + i) * NB + c] = acc;
  }
}

__global__ __launch_bounds__(64) void k_ir_resid_sum(const BackBatch B) {
  int q = 0;
  while (q + 1 < B.nprob && (int)blockIdx.x >= B.wg0[q + 1]) q++;
  const CholArgs& P = B.p[q];
  const int nb = P.nb, i = (int)blockIdx.x - B.wg0[q], r = threadIdx.x;
  const double* part = P.xd + P.npad + (size_t)i * nb * NB;
  double acc = 0.0;
#pragma unroll 8
  for (int k = 0; k < nb; k++) acc += part[(size_t)k * NB + r];
  const size_t gi = (size_t)NB * i + r;
  P.A[(size_t)P.npad * P.ld + gi] = (float)((double)P.c[gi] - (double)P.dscale[gi] * acc);
}

// A0 = the lower-triangle tiles of the damped matrix A (the only part the residual reads), before
// the factorisation overwrites them, one workgroup per tile; the workgroup of diagonal tile i also
// keeps block i of the equilibrated right-hand side (row npad of A) in c.
__global__ __launch_bounds__(256) void k_ir_copy_lower(const BackBatch B) {
  int t = (int)blockIdx.x;
  const CholArgs& P = B.p[lower_tile_system(B, t)];
  int i, k;
  lower_tile_of(t, i, k);
#pragma unroll
  for (int u = 0; u < 4; u++) {
    const int e = threadIdx.x + 256 * u, r = e >> 4, c = 4 * (e & 15);
    const size_t o = (size_t)(NB * i + r) * P.ld + NB * k + c;
    *reinterpret_cast<float4*>(const_cast<float*>(P.A0) + o) = *reinterpret_cast<const float4*>(P.A + o);
  }
  if (i == k && threadIdx.x < NB) {
    const size_t gi = (size_t)NB * i + threadIdx.x;
    const_cast<float*>(P.c)[gi] = P.A[(size_t)P.npad * P.ld + gi];
  }
}

// xd = x (mode 0), or xd += x and x = xd rounded (mode 1). One wavefront per block of 64 entries.
__global__ __launch_bounds__(64) void k_ir_accum(const BackBatch B, int mode) {
  int q = 0;
  while (q + 1 < B.nprob && (int)blockIdx.x >= B.wg0[q + 1]) q++;
  const CholArgs& P = B.p[q];
  const size_t i = (size_t)NB * ((int)blockIdx.x - B.wg0[q]) + threadIdx.x;
  if (mode == 0) {
    P.xd[i] = (double)P.x[i];
  } else {
    const double v = P.xd[i] + (double)P.x[i];
    P.xd[i] = v;
    P.x[i] = (float)v;
  }
}

}  // namespace

size_t chol_flag_ints(int nb) { return (size_t)nb + (size_t)(nb + 1) * nb + 4 * (size_t)nb + 2; }

static CholArgs chol_args(const DevState& d, int which) {
  CholArgs P;
  P.A = d.A;
  P.ld = d.ld;
  P.npad = d.npad;
  P.nb = d.nb;
  P.ntasks = chol_task_count(d.nb);
  P.which = which;
  P.dscale = d.dscale;
  P.Linv = d.Linv;
  P.flags = d.flags;
  P.sc = d.sc;
  P.x = d.x;
  P.prec = d.prec;
  P.A16 = d.A16;
  P.A0 = d.A0;
  P.c = d.cvec;
  P.xd = d.xd;
  P.tw = d.tw;
  return P;
}

// A hand-over wait of the factorisation gives up after this long (then the step is rejected and
// the failure reported): far beyond any wait of a working solve, short enough to end a broken one.
constexpr double kWaitSeconds = 1.0;

hipError_t launch_cholesky_factor_batch(DevState* const* ds, int S, hipStream_t st) {
  for (int b0 = 0; b0 < S; b0 += kMaxCholBatch) {
    CholBatch B;
    B.nprob = (S - b0 < kMaxCholBatch) ? S - b0 : kMaxCholBatch;
    int tasks = 0, cus = 256, khz = 100000;  // the constant clock runs at 100 MHz unless the device says otherwise
    // launch width in percent of the compute units: the widest of the systems' tunings (a batch
    // holds at least the work of its largest system)
    int pct = 0;
    for (int q = 0; q < B.nprob; q++) {
      B.p[q] = chol_args(*ds[b0 + q], 0);
      tasks += B.p[q].ntasks;
      if (ds[b0 + q]->num_cus > 0) cus = ds[b0 + q]->num_cus;
      if (ds[b0 + q]->wall_khz > 0) khz = ds[b0 + q]->wall_khz;
      const int t = ds[b0 + q]->chol_grid_pct;
      if (t >= 25 && t <= 400 && t > pct) pct = t;
    }
    if (pct == 0) pct = 200;
    B.wait_ticks = (uint64_t)(kWaitSeconds * 1000.0 * khz);
    // any width is safe: a task waits only on smaller tickets, which running workgroups claimed
    const int width = (cus * pct + 99) / 100;
    const int grid = tasks < width ? tasks : width;
    hipLaunchKernelGGL(k_chol_dataflow, dim3(grid), dim3(256), 0, st, B);
  }
  return hipGetLastError();
}

hipError_t launch_cholesky_factor(DevState& d, hipStream_t st) {
  DevState* ds[1] = {&d};
  return launch_cholesky_factor_batch(ds, 1, st);
}

// One launch per (up to) 32 systems of a per-block-row kernel (grid: 64-row blocks of every system).
template <typename F>
static hipError_t launch_rows_batch(DevState* const* ds, int which, int S, F launch) {
  for (int b0 = 0; b0 < S; b0 += kMaxCholBatch) {
    BackBatch B;
    B.nprob = (S - b0 < kMaxCholBatch) ? S - b0 : kMaxCholBatch;
    B.wg0[0] = 0;
    for (int q = 0; q < B.nprob; q++) {
      B.p[q] = chol_args(*ds[b0 + q], which);
      B.wg0[q + 1] = B.wg0[q] + ds[b0 + q]->nb;
    }
    launch(B);
  }
  return hipGetLastError();
}

hipError_t launch_cholesky_backsolve_batch(DevState* const* ds, int which, int S, hipStream_t st) {
  return launch_rows_batch(ds, which, S, [&](const BackBatch& B) {
    hipLaunchKernelGGL(k_chol_backsolve, dim3(B.wg0[B.nprob]), dim3(64), 0, st, B);
  });
}

hipError_t launch_cholesky_backsolve(DevState& d, int which, hipStream_t st) {
  DevState* ds[1] = {&d};
  return launch_cholesky_backsolve_batch(ds, which, 1, st);
}

static int lower_tiles(const BackBatch& B) {
  int n = 0;
  for (int q = 0; q < B.nprob; q++) n += B.p[q].nb * (B.p[q].nb + 1) / 2;
  return n;
}

hipError_t launch_ir_prepare_batch(DevState* const* ds, int S, hipStream_t st) {
  return launch_rows_batch(ds, 0, S, [&](const BackBatch& B) {
    hipLaunchKernelGGL(k_ir_copy_lower, dim3(lower_tiles(B)), dim3(256), 0, st, B);
  });
}

hipError_t launch_ir_prepare(DevState& d, hipStream_t st) {
  DevState* ds[1] = {&d};
  return launch_ir_prepare_batch(ds, 1, st);
}

hipError_t launch_ir_step_batch(DevState* const* ds, int step, int S, hipStream_t st) {
  hipError_t e = launch_rows_batch(ds, 0, S, [&](const BackBatch& B) {
    hipLaunchKernelGGL(k_ir_resid_tiles, dim3(lower_tiles(B)), dim3(256), 0, st, B);
    hipLaunchKernelGGL(k_ir_resid_sum, dim3(B.wg0[B.nprob]), dim3(64), 0, st, B);
  });
  if (e != hipSuccess) return e;
  e = launch_rows_batch(ds, 1 + 2 * step, S, [&](const BackBatch& B) {
    hipLaunchKernelGGL(k_chol_fwdsolve, dim3(B.wg0[B.nprob]), dim3(64), 0, st, B);
  });
  if (e != hipSuccess) return e;
  e = launch_cholesky_backsolve_batch(ds, 2 + 2 * step, S, st);
  if (e != hipSuccess) return e;
  return launch_ir_accum_batch(ds, S, 1, st);
}

hipError_t launch_ir_accum_batch(DevState* const* ds, int S, int mode, hipStream_t st) {
  return launch_rows_batch(ds, 0, S, [&](const BackBatch& B) {
    hipLaunchKernelGGL(k_ir_accum, dim3(B.wg0[B.nprob]), dim3(64), 0, st, B, mode);
  });
}
