// tt_orb.hip -- uniform ORB features on gfx950 (Sec. 2.1): FAST corners computed for every pixel
// in parallel, kept where no neighbouring pixel has a larger corner response, then oriented
// binary descriptors and 3D points from the depth map.
//
//   k_orb_box5      5x5 box sums of the image (the smoothed image the descriptor tests compare)
//   k_orb_response  FAST-9 response of every pixel of the detection region (0: not a corner)
//   k_orb_nms       one workgroup per row: suppression against the (2r+1)^2 window, row counts
//   k_orb_scan      exclusive scan of the row counts (one workgroup)
//   k_orb_emit      one workgroup per row: the row's kept pixels in raster order, capped
//   k_orb_describe  one wavefront per keypoint: intensity-centroid orientation (integer moments,
//                   wave reduction), 256 tests on the rotated pattern, depth back-projection
//
// Keypoints come out in raster order, so the result does not depend on the launch shape; every
// decision is integer except the orientation bin, which is taken in FP64 from exact integer
// moments.
#include <math.h>
#include <string.h>

#include <mutex>
#include <new>
#include <vector>

#include "tt_internal.h"

namespace {

constexpr int kBorder = 18;  // FAST circle 3, orientation disc 15, rotated pattern + box 16

__constant__ int2 kCircle[16] = {{0, -3}, {1, -3}, {2, -2}, {3, -1}, {3, 0}, {3, 1}, {2, 2}, {1, 3},
                                 {0, 3}, {-1, 3}, {-2, 2}, {-3, 1}, {-3, 0}, {-3, -1}, {-2, -2}, {-1, -3}};

__global__ void k_orb_box5(const uint8_t* __restrict__ img, int W, int H, int* __restrict__ S) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x, v = blockIdx.y;
  if (u >= W) return;
  int acc = 0;
  if (u >= 2 && u < W - 2 && v >= 2 && v < H - 2) {
#pragma unroll
    for (int dy = -2; dy <= 2; dy++)
#pragma unroll
      for (int dx = -2; dx <= 2; dx++) acc += img[(size_t)(v + dy) * W + u + dx];
  }
  S[(size_t)v * W + u] = acc;
}

// 9 or more contiguous set bits (cyclic) in a 16-bit circle mask
__device__ __forceinline__ bool run9(unsigned m) {
  unsigned x = m | (m << 16);
  unsigned a = x;
#pragma unroll
  for (int s = 1; s < 9; s++) a &= x >> s;
  return a != 0;
}

__global__ void k_orb_response(const uint8_t* __restrict__ img, int W, int H, int t, int* __restrict__ R) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x, v = blockIdx.y;
  if (u >= W) return;
  int resp = 0;
  if (u >= kBorder && u < W - kBorder && v >= kBorder && v < H - kBorder) {
    const int c = img[(size_t)v * W + u];
    unsigned mb = 0, md = 0;
    int sb = 0, sd = 0;
#pragma unroll
    for (int k = 0; k < 16; k++) {
      const int x = img[(size_t)(v + kCircle[k].y) * W + u + kCircle[k].x];
      if (x > c + t) {
        mb |= 1u << k;
        sb += x - c - t;
      } else if (x < c - t) {
        md |= 1u << k;
        sd += c - x - t;
      }
    }
    if (run9(mb) || run9(md)) resp = sb > sd ? sb : sd;
  }
  R[(size_t)v * W + u] = resp;
}

constexpr int kRowThreads = 256;

// kept iff no other corner of the window has a larger response, ties to the lower pixel index
__device__ __forceinline__ bool orb_keep(const int* __restrict__ R, int W, int H, int u, int v, int r) {
  const size_t i = (size_t)v * W + u;
  const int Ri = R[i];
  if (Ri <= 0) return false;
  for (int dy = -r; dy <= r; dy++) {
    const int vv = v + dy;
    if (vv < 0 || vv >= H) continue;
    for (int dx = -r; dx <= r; dx++) {
      const int uu = u + dx;
      if ((dx == 0 && dy == 0) || uu < 0 || uu >= W) continue;
      const size_t q = (size_t)vv * W + uu;
      const int Rq = R[q];
      if (Rq > Ri || (Rq == Ri && q < i)) return false;
    }
  }
  return true;
}

__global__ __launch_bounds__(kRowThreads) void k_orb_nms(const int* __restrict__ R, int W, int H, int r,
                                                         uint8_t* __restrict__ flags, int* __restrict__ rowcnt) {
  __shared__ int wsum[kRowThreads / 64];
  const int v = blockIdx.x;
  int cnt = 0;
  for (int u = threadIdx.x; u < W; u += kRowThreads) {
    const bool k = orb_keep(R, W, H, u, v, r);
    flags[(size_t)v * W + u] = k ? 1 : 0;
    cnt += k ? 1 : 0;
  }
  // integer sum: order does not matter
  for (int s = 32; s > 0; s >>= 1) cnt += __shfl_xor(cnt, s);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < kRowThreads / 64; w++) t += wsum[w];
    rowcnt[v] = t;
  }
}

constexpr int kScanThreads = 1024;

// exclusive scan of H row counts; count[0] = min(total, cap), count[1] = total
__global__ __launch_bounds__(kScanThreads) void k_orb_scan(const int* __restrict__ rowcnt, int H, int cap,
                                                           int* __restrict__ rowoff, int32_t* __restrict__ count) {
  __shared__ int sh[kScanThreads];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < H; base += kScanThreads) {
    const int i = base + threadIdx.x;
    const int x = i < H ? rowcnt[i] : 0;
    sh[threadIdx.x] = x;
    __syncthreads();
    for (int s = 1; s < kScanThreads; s <<= 1) {  // inclusive Hillis-Steele scan
      const int y = threadIdx.x >= s ? sh[threadIdx.x - s] : 0;
      __syncthreads();
      sh[threadIdx.x] += y;
      __syncthreads();
    }
    if (i < H) rowoff[i] = carry + sh[threadIdx.x] - x;
    __syncthreads();
    if (threadIdx.x == kScanThreads - 1) carry += sh[kScanThreads - 1];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    count[0] = carry < cap ? carry : cap;
    count[1] = carry;
  }
}

__global__ __launch_bounds__(kRowThreads) void k_orb_emit(const uint8_t* __restrict__ flags, int W,
                                                          const int* __restrict__ rowoff, int cap,
                                                          int32_t* __restrict__ kp) {
  __shared__ int woff[kRowThreads / 64 + 1];
  const int v = blockIdx.x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int base = rowoff[v];
  for (int u0 = 0; u0 < W; u0 += kRowThreads) {
    const int u = u0 + threadIdx.x;
    const bool f = u < W && flags[(size_t)v * W + u];
    const unsigned long long m = __ballot(f);
    const int before = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) woff[w] = __popcll(m);
    __syncthreads();
    int off = 0;
    for (int q = 0; q < w; q++) off += woff[q];
    int chunk = 0;
    for (int q = 0; q < kRowThreads / 64; q++) chunk += woff[q];
    const int slot = base + off + before;
    if (f && slot < cap) {
      kp[2 * slot] = u;
      kp[2 * slot + 1] = v;
    }
    base += chunk;
    __syncthreads();
  }
}

struct OrbIntr {
  double fx, fy, cx, cy;
};

// One wavefront per keypoint.
__global__ __launch_bounds__(64) void k_orb_describe(const uint8_t* __restrict__ img, const int* __restrict__ S, int W,
                                                     const int32_t* __restrict__ count, const int32_t* __restrict__ kp,
                                                     const int8_t* __restrict__ rotpat, const float* __restrict__ depth,
                                                     OrbIntr K, float* __restrict__ xyz, uint8_t* __restrict__ desc,
                                                     int32_t* __restrict__ angle) {
  const int n = blockIdx.x;
  if (n >= count[0]) return;  // the whole wavefront: keypoints beyond the count
  const int lane = threadIdx.x;
  const int u = kp[2 * n], v = kp[2 * n + 1];
  // intensity centroid over the disc of radius 15
  int m10 = 0, m01 = 0;
  for (int o = lane; o < 31 * 31; o += 64) {
    const int dy = o / 31 - 15, dx = o % 31 - 15;
    if (dx * dx + dy * dy > 225) continue;
    const int I = img[(size_t)(v + dy) * W + u + dx];
    m10 += dx * I;
    m01 += dy * I;
  }
  for (int s = 32; s > 0; s >>= 1) {
    m10 += __shfl_xor(m10, s);
    m01 += __shfl_xor(m01, s);
  }
  const double th = atan2((double)m01, (double)m10);
  int bin = (int)floor(th * 30.0 / (2.0 * 3.14159265358979323846) + 0.5);
  bin = ((bin % 30) + 30) % 30;
  // four tests per lane: pattern pairs 4 lane .. 4 lane + 3
  const char4* rp = reinterpret_cast<const char4*>(rotpat) + (size_t)bin * 256;
  unsigned nib = 0;
#pragma unroll
  for (int q = 0; q < 4; q++) {
    const char4 pr = rp[4 * lane + q];
    const int sa = S[(size_t)(v + pr.y) * W + u + pr.x];
    const int sb = S[(size_t)(v + pr.w) * W + u + pr.z];
    nib |= (sa < sb ? 1u : 0u) << q;
  }
  const unsigned hi = __shfl_down(nib, 1);
  if ((lane & 1) == 0) desc[32 * (size_t)n + (lane >> 1)] = (uint8_t)(nib | (hi << 4));
  if (lane == 0) {
    if (angle) angle[n] = bin;
    if (xyz) {
      const float z = depth ? depth[(size_t)v * W + u] : NAN;
      float* o = xyz + 3 * (size_t)n;
      if (depth && isfinite(z) && z > 0.0f) {
        o[0] = (float)(((double)u - K.cx) / K.fx * (double)z);
        o[1] = (float)(((double)v - K.cy) / K.fy * (double)z);
        o[2] = z;
      } else {
        o[0] = o[1] = o[2] = NAN;
      }
    }
  }
}

}  // namespace

struct tt_orb {
  std::mutex mu;  // one call at a time (the working buffers are the detector's)
  tt_orb_params P;
  int W = 0, H = 0;
  hipStream_t st = nullptr;
  bool own_stream = false;
  int* R = nullptr;
  int* S = nullptr;
  uint8_t* flags = nullptr;
  int* rowcnt = nullptr;
  int* rowoff = nullptr;
  int8_t* rotpat = nullptr;
  // staging for the host entry point
  uint8_t* img = nullptr;
  float* depth = nullptr;
  int32_t* kp = nullptr;
  float* xyz = nullptr;
  uint8_t* desc = nullptr;
  int32_t* angle = nullptr;
  int32_t* count = nullptr;
};

namespace {

struct OrbBusy {
  tt_orb* o;
  bool ok;
  explicit OrbBusy(tt_orb* o_) : o(o_), ok(o_->mu.try_lock()) {}
  ~OrbBusy() {
    if (ok) o->mu.unlock();
  }
};

void orb_free(tt_orb* o) {
  void* ps[] = {o->R, o->S, o->flags, o->rowcnt, o->rowoff, o->rotpat, o->img, o->depth, o->kp, o->xyz, o->desc,
                o->angle, o->count};
  for (void* p : ps)
    if (p) (void)hipFree(p);
}

int orb_enqueue(tt_orb* o, const uint8_t* img, const float* depth, const tt_intrinsics* K, int32_t* kp, float* xyz,
                uint8_t* desc, int32_t* angle, int32_t* count) {
  const int W = o->W, H = o->H;
  hipStream_t st = o->st;
  const dim3 rows((W + kRowThreads - 1) / kRowThreads, H);
  hipLaunchKernelGGL(k_orb_box5, rows, dim3(kRowThreads), 0, st, img, W, H, o->S);
  hipLaunchKernelGGL(k_orb_response, rows, dim3(kRowThreads), 0, st, img, W, H, o->P.fast_threshold, o->R);
  hipLaunchKernelGGL(k_orb_nms, dim3(H), dim3(kRowThreads), 0, st, o->R, W, H, o->P.nms_radius, o->flags, o->rowcnt);
  hipLaunchKernelGGL(k_orb_scan, dim3(1), dim3(kScanThreads), 0, st, o->rowcnt, H, o->P.max_features, o->rowoff,
                     count);
  hipLaunchKernelGGL(k_orb_emit, dim3(H), dim3(kRowThreads), 0, st, o->flags, W, o->rowoff, o->P.max_features, kp);
  OrbIntr ki{1.0, 1.0, 0.0, 0.0};
  if (K) ki = OrbIntr{K->fx, K->fy, K->cx, K->cy};
  if (o->P.max_features > 0)
    hipLaunchKernelGGL(k_orb_describe, dim3(o->P.max_features), dim3(64), 0, st, img, o->S, W, count, kp, o->rotpat,
                       depth, ki, xyz, desc, angle);
  return hipGetLastError() == hipSuccess ? TT_OK : TT_EDEVICE;
}

}  // namespace

extern "C" {

void tt_orb_default_params(tt_orb_params* p) {
  if (!p) return;
  p->fast_threshold = 20;
  p->nms_radius = 1;
  p->max_features = 4096;
}

int tt_orb_create(const tt_orb_params* p, int width, int height, const int8_t* pattern, void* hip_stream,
                  tt_orb** out) {
  if (!p || !pattern || !out) return TT_EINVAL;
  *out = nullptr;
  if (width < 1 || height < 1 || (int64_t)width * height > (1 << 28) || p->fast_threshold < 0 ||
      p->fast_threshold > 255 || p->nms_radius < 0 || p->nms_radius > 16 || p->max_features < 0 ||
      p->max_features > (1 << 20))
    return TT_EINVAL;
  for (int k = 0; k < 256; k++)
    for (int h = 0; h < 2; h++) {
      const int x = pattern[4 * k + 2 * h], y = pattern[4 * k + 2 * h + 1];
      if (x * x + y * y > 169) return TT_EINVAL;  // the border assumes offsets within radius 13
    }
  tt_orb* o = new (std::nothrow) tt_orb();
  if (!o) return TT_ENOMEM;
  o->P = *p;
  o->W = width;
  o->H = height;
  if (hip_stream) {
    o->st = static_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreateWithFlags(&o->st, hipStreamNonBlocking) != hipSuccess) {
      delete o;
      return TT_EDEVICE;
    }
    o->own_stream = true;
  }
  // the pattern rotated to each of the 30 orientation bins (12 degrees apart), rounded half away
  // from zero
  std::vector<int8_t> rot(30 * 256 * 4);
  for (int b = 0; b < 30; b++) {
    const double th = 2.0 * 3.14159265358979323846 * b / 30.0, cs = cos(th), sn = sin(th);
    for (int k = 0; k < 256; k++)
      for (int h = 0; h < 2; h++) {
        const double x = pattern[4 * k + 2 * h], y = pattern[4 * k + 2 * h + 1];
        rot[(size_t)(b * 256 + k) * 4 + 2 * h] = (int8_t)lround(x * cs - y * sn);
        rot[(size_t)(b * 256 + k) * 4 + 2 * h + 1] = (int8_t)lround(x * sn + y * cs);
      }
  }
  const size_t HW = (size_t)width * height, mx = p->max_features > 0 ? (size_t)p->max_features : 1;
  bool ok = hipMalloc((void**)&o->R, sizeof(int) * HW) == hipSuccess &&
            hipMalloc((void**)&o->S, sizeof(int) * HW) == hipSuccess &&
            hipMalloc((void**)&o->flags, HW) == hipSuccess &&
            hipMalloc((void**)&o->rowcnt, sizeof(int) * height) == hipSuccess &&
            hipMalloc((void**)&o->rowoff, sizeof(int) * height) == hipSuccess &&
            hipMalloc((void**)&o->rotpat, rot.size()) == hipSuccess &&
            hipMalloc((void**)&o->img, HW) == hipSuccess && hipMalloc((void**)&o->depth, sizeof(float) * HW) == hipSuccess &&
            hipMalloc((void**)&o->kp, sizeof(int32_t) * 2 * mx) == hipSuccess &&
            hipMalloc((void**)&o->xyz, sizeof(float) * 3 * mx) == hipSuccess &&
            hipMalloc((void**)&o->desc, 32 * mx) == hipSuccess &&
            hipMalloc((void**)&o->angle, sizeof(int32_t) * mx) == hipSuccess &&
            hipMalloc((void**)&o->count, sizeof(int32_t) * 2) == hipSuccess;
  ok = ok && hipMemcpy(o->rotpat, rot.data(), rot.size(), hipMemcpyHostToDevice) == hipSuccess;
  if (!ok) {
    orb_free(o);
    if (o->own_stream) (void)hipStreamDestroy(o->st);
    delete o;
    return TT_ENOMEM;
  }
  *out = o;
  return TT_OK;
}

int tt_orb_detect_device(tt_orb* o, const uint8_t* d_image, const float* d_depth, const tt_intrinsics* K,
                         int32_t* d_kp, float* d_xyz, uint8_t* d_desc, int32_t* d_angle, int32_t* d_count) {
  if (!o || !d_image || !d_count || (d_depth && !K) || (o->P.max_features > 0 && (!d_kp || !d_desc)))
    return TT_EINVAL;
  if (K && (K->width != o->W || K->height != o->H || !(K->fx > 0) || !(K->fy > 0))) return TT_EINVAL;
  OrbBusy busy(o);
  if (!busy.ok) return TT_EBUSY;
  return orb_enqueue(o, d_image, d_depth, K, d_kp, d_xyz, d_desc, d_angle, d_count);
}

int tt_orb_detect(tt_orb* o, const uint8_t* image, const float* depth, const tt_intrinsics* K, int32_t* kp,
                  float* xyz, uint8_t* desc, int32_t* angle, int32_t* count) {
  if (!o || !image || !count || (depth && !K) || (o->P.max_features > 0 && (!kp || !desc))) return TT_EINVAL;
  if (K && (K->width != o->W || K->height != o->H || !(K->fx > 0) || !(K->fy > 0))) return TT_EINVAL;
  OrbBusy busy(o);
  if (!busy.ok) return TT_EBUSY;
  const size_t HW = (size_t)o->W * o->H;
  hipStream_t st = o->st;
  if (hipMemcpyAsync(o->img, image, HW, hipMemcpyHostToDevice, st) != hipSuccess) return TT_EDEVICE;
  if (depth && hipMemcpyAsync(o->depth, depth, sizeof(float) * HW, hipMemcpyHostToDevice, st) != hipSuccess)
    return TT_EDEVICE;
  int rc = orb_enqueue(o, o->img, depth ? o->depth : nullptr, K, o->kp, o->xyz, o->desc, o->angle, o->count);
  if (rc) return rc;
  int32_t c[2] = {0, 0};
  if (hipMemcpyAsync(c, o->count, sizeof(c), hipMemcpyDeviceToHost, st) != hipSuccess) return TT_EDEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) return TT_EDEVICE;
  const size_t n = (size_t)c[0];
  bool ok = true;
  if (n) {
    ok = ok && hipMemcpyAsync(kp, o->kp, sizeof(int32_t) * 2 * n, hipMemcpyDeviceToHost, st) == hipSuccess;
    ok = ok && hipMemcpyAsync(desc, o->desc, 32 * n, hipMemcpyDeviceToHost, st) == hipSuccess;
    if (xyz) ok = ok && hipMemcpyAsync(xyz, o->xyz, sizeof(float) * 3 * n, hipMemcpyDeviceToHost, st) == hipSuccess;
    if (angle) ok = ok && hipMemcpyAsync(angle, o->angle, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st) == hipSuccess;
  }
  ok = ok && hipStreamSynchronize(st) == hipSuccess;
  count[0] = c[0];
  count[1] = c[1];
  return ok ? TT_OK : TT_EDEVICE;
}

void* tt_orb_hip_stream(tt_orb* o) { return o ? static_cast<void*>(o->st) : nullptr; }

int tt_orb_destroy(tt_orb* o) {
  if (!o) return TT_EINVAL;
  {
    OrbBusy busy(o);
    if (!busy.ok) return TT_EBUSY;
  }
  (void)hipStreamSynchronize(o->st);
  orb_free(o);
  if (o->own_stream) (void)hipStreamDestroy(o->st);
  delete o;
  return TT_OK;
}

}  // extern "C"
