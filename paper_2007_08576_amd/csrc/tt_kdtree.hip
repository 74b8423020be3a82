// tt_kdtree.hip -- per-frame kd-tree of the frame's points for the closest-point association
// comparator (assoc_kdtree; the paper's re-projection replaces this search, Sec. 2).
//
// Build, all on the device and with no host round trip (the number of points P is known only on the
// device, so every pass runs over all H*W slots and reads P from memory):
//   1. flag the pixels that have a normal; ordered compaction of their indices (hipCUB select, stable)
//      and their float32 back-projections;
//   2. for each depth t = 0 .. levels - 1: key every position i < P by (its node at depth t, the
//      float32 coordinate on that depth's axis, order-preserving bits) and every slot i >= P past all
//      nodes; one stable radix sort of (key, point) pairs; then every node of depth t records the
//      coordinate at its midpoint as its split value. Each node's positions are thereby sorted on its
//      axis, so its lower half holds the smaller coordinates -- the halves are the children;
//   3. gather the points (x, y, z, pixel) in tree order.
// Ties keep the order of the previous pass (stable sort), so the tree is deterministic.
#include <hipcub/hipcub.hpp>

#include "tt_internal.h"

namespace {

constexpr int kT = 256;

__global__ void k_kd_flag(const float4* __restrict__ nmap, int HW, uint8_t* __restrict__ flag) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i < HW) {
    const float4 n = nmap[i];
    flag[i] = (n.x != 0.0f || n.y != 0.0f || n.z != 0.0f) ? 1 : 0;
  }
}

// float32 back-projection of the selected pixels, ((u - cx) / fx z, (v - cy) / fy z, z) in FP64 rounded
// once; vals = identity
__global__ void k_kd_points(const int* __restrict__ sel, const int* __restrict__ count, const float* __restrict__ depth,
                            int W, double fx, double fy, double cx, double cy, int HW, float4* __restrict__ xyz,
                            uint32_t* __restrict__ vals) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i >= HW) return;
  vals[i] = (uint32_t)i;
  if (i < *count) {
    const int pix = sel[i];
    const double z = depth[pix];
    const double u = pix % W, v = pix / W;
    xyz[i] = make_float4((float)((u - cx) / fx * z), (float)((v - cy) / fy * z), (float)z, __int_as_float(pix));
  }
}

// order-preserving unsigned bits of a float (negative values reversed)
__device__ __forceinline__ uint32_t sortable(float f) {
  const uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// node (within its depth) of position i < P at depth t
__device__ __forceinline__ uint32_t node_of(int i, int P, int t) {
  int lo = 0, hi = P;
  uint32_t k = 0;
  for (int s = 0; s < t; s++) {
    const int mid = lo + (hi - lo) / 2;
    if (i < mid) {
      hi = mid;
      k = 2 * k;
    } else {
      lo = mid;
      k = 2 * k + 1;
    }
  }
  return k;
}

__global__ void k_kd_keys(const float4* __restrict__ xyz, const uint32_t* __restrict__ vals, const int* __restrict__ count,
                          int HW, int t, uint64_t* __restrict__ keys) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i >= HW) return;
  const int P = *count;
  if (i < P) {
    const float4 p = xyz[vals[i]];
    keys[i] = ((uint64_t)node_of(i, P, t) << 32) | sortable((t & 1) ? p.y : p.x);
  } else {
    keys[i] = (uint64_t)(1u << t) << 32;  // past every node of depth t
  }
}

__global__ void k_kd_split(const float4* __restrict__ xyz, const uint32_t* __restrict__ vals, const int* __restrict__ count,
                           int t, float* __restrict__ split) {
  const int k = blockIdx.x * kT + threadIdx.x;
  if (k >= (1 << t)) return;
  const int P = *count;
  int lo = 0, hi = P;
  for (int s = t - 1; s >= 0; s--) {
    const int mid = lo + (hi - lo) / 2;
    if ((k >> s) & 1) lo = mid;
    else hi = mid;
  }
  float v = 0.0f;
  if (hi > lo) {
    const float4 p = xyz[vals[lo + (hi - lo) / 2]];
    v = (t & 1) ? p.y : p.x;
  }
  split[(1 << t) + k] = v;
}

__global__ void k_kd_gather(const float4* __restrict__ xyz, const uint32_t* __restrict__ vals, const int* __restrict__ count,
                            int HW, float4* __restrict__ pts) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i < HW && i < *count) pts[i] = xyz[vals[i]];
}

}  // namespace

int kd_levels_for(int HW) {
  int L = 0;
  while (L < 28 && ((int64_t)HW >> L) > kKdLeaf) L++;
  return L;
}

size_t kd_scratch_bytes(int HW) {
  size_t a = 0, b = 0;
  hipcub::DoubleBuffer<uint64_t> dk(nullptr, nullptr);
  hipcub::DoubleBuffer<uint32_t> dv(nullptr, nullptr);
  if (hipcub::DeviceRadixSort::SortPairs(nullptr, a, dk, dv, HW, 0, 64, (hipStream_t)0) != hipSuccess) return 0;
  if (hipcub::DeviceSelect::Flagged(nullptr, b, hipcub::CountingInputIterator<int>(0), (const uint8_t*)nullptr,
                                    (int*)nullptr, (int*)nullptr, HW, (hipStream_t)0) != hipSuccess)
    return 0;
  return a > b ? a : b;
}

hipError_t launch_kd_build(DevState& d, const Intr& K, hipStream_t st) {
  const int HW = d.HW, L = d.kd_levels;
  const dim3 g((HW + kT - 1) / kT);
  hipLaunchKernelGGL(k_kd_flag, g, dim3(kT), 0, st, d.nmap, HW, d.kd_flag);
  size_t bytes = d.kd_temp_bytes;
  hipError_t e = hipcub::DeviceSelect::Flagged(d.kd_temp, bytes, hipcub::CountingInputIterator<int>(0), d.kd_flag,
                                               d.kd_sel, d.kd_count, HW, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_kd_points, g, dim3(kT), 0, st, d.kd_sel, d.kd_count, d.depth, K.W, K.fx, K.fy, K.cx, K.cy, HW,
                     d.kd_xyz, d.kd_vals);
  hipcub::DoubleBuffer<uint64_t> dk(d.kd_keys, d.kd_keys + HW);
  hipcub::DoubleBuffer<uint32_t> dv(d.kd_vals, d.kd_vals + HW);
  for (int t = 0; t < L; t++) {
    hipLaunchKernelGGL(k_kd_keys, g, dim3(kT), 0, st, d.kd_xyz, dv.Current(), d.kd_count, HW, t, dk.Current());
    bytes = d.kd_temp_bytes;
    // node bits 32 .. 32 + t (the slots past every node use bit 32 + t)
    e = hipcub::DeviceRadixSort::SortPairs(d.kd_temp, bytes, dk, dv, HW, 0, 33 + t, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_kd_split, dim3(((1 << t) + kT - 1) / kT), dim3(kT), 0, st, d.kd_xyz, dv.Current(), d.kd_count,
                       t, d.kd_split);
  }
  hipLaunchKernelGGL(k_kd_gather, g, dim3(kT), 0, st, d.kd_xyz, dv.Current(), d.kd_count, HW, d.kd_pts);
  return hipGetLastError();
}
