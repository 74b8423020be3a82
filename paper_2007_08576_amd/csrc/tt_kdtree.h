// tt_kdtree.h -- nearest frame point of a deformed template point through a kd-tree: the
// closest-point association that the paper names as the slower alternative to its re-projection
// ("rasterization", Sec. 2). Device side of the query; the tree is built per frame by
// launch_kd_build (tt_kdtree.hip).
//
// Tree: the frame's points (back-projected pixels that have a normal, float32) in tree order. The
// node of depth t covering positions [lo, hi) of [0, P) splits at mid = lo + (hi - lo) / 2 on x
// (t even) or y (t odd) -- the back-projected depth is a height field over the image plane, so the
// splits alternate between its two spread-out axes while distances stay three-dimensional; the
// points of [lo, mid) have coordinates <= split[node], those of [mid, hi) >= it (heap order,
// root 1, children 2 node and 2 node + 1). Nodes of depth `levels` are leaves, searched whole.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

struct KdArgs {
  const float4* pts;   // [P] x, y, z, pixel index (int bits)
  const float* split;  // [2^levels] split value of each internal node (index 1 .. 2^levels - 1)
  const int* count;    // P, written by the build
  int levels;
};

// Squared distance in the fixed order (dx^2 + dy^2) + dz^2 with no contraction, so that a node's
// squared split gap (the first or second term alone) never exceeds the computed squared distance
// of a point behind the split, and pruning with it is exact for these distances.
__device__ __forceinline__ float kd_d2(float4 p, float vx, float vy, float vz) {
  const float dx = __fsub_rn(p.x, vx), dy = __fsub_rn(p.y, vy), dz = __fsub_rn(p.z, vz);
  return __fadd_rn(__fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy)), __fmul_rn(dz, dz));
}

// Positions [lo, hi) covered by node (depth d): the halvings from the root along its bits.
__device__ __forceinline__ void kd_range(int node, int d, int P, int& lo, int& hi) {
  lo = 0;
  hi = P;
  for (int s = d - 1; s >= 0; s--) {
    const int mid = lo + (hi - lo) / 2;
    if ((node >> s) & 1) lo = mid;
    else hi = mid;
  }
}

// Pixel of the nearest point by float32 squared distance (ties: the lower pixel index), -1 if the
// frame has no point. Depth-first, near child first; a far child is visited unless its split gap
// squared exceeds the best distance so far (equal gaps are visited, for the tie rule). No stack:
// bit t of `pend` marks that the current path took the near child at depth t while the far child
// is not empty and was not pruned when the path passed; after a leaf the search resumes at the
// deepest marked depth (the gap is recomputed from the split and checked again, the far child's
// range recomputed from its node index), which visits the far children deepest first, as a stack
// of them would.
__device__ __forceinline__ int kd_nearest(const KdArgs& kd, float vx, float vy, float vz) {
  const int P = *kd.count;
  if (P <= 0) return -1;
  float best = __builtin_huge_valf();
  int bpix = 0x7fffffff;
  int node = 1, depth = 0, lo = 0, hi = P;
  uint32_t pend = 0;
  for (;;) {
    while (depth < kd.levels) {
      const int mid = lo + (hi - lo) / 2;
      const float diff = __fsub_rn((depth & 1) ? vy : vx, kd.split[node]);
      const bool far_nonempty = (diff < 0.0f) ? (mid < hi) : (lo < mid);
      if (far_nonempty && __fmul_rn(diff, diff) <= best) pend |= 1u << depth;
      if (diff < 0.0f) {  // near: the lower half
        hi = mid;
        node = 2 * node;
      } else {
        lo = mid;
        node = 2 * node + 1;
      }
      depth += 1;
    }
    for (int i = lo; i < hi; i++) {
      const float4 p = kd.pts[i];
      const float d2 = kd_d2(p, vx, vy, vz);
      const int pix = __float_as_int(p.w);
      if (d2 < best || (d2 == best && pix < bpix)) {
        best = d2;
        bpix = pix;
      }
    }
    bool down = false;
    while (pend != 0u && !down) {
      const int t = 31 - __builtin_clz(pend);
      pend &= ~(1u << t);
      const int parent = node >> (depth - t);
      const float diff = __fsub_rn((t & 1) ? vy : vx, kd.split[parent]);
      if (__fmul_rn(diff, diff) > best) continue;
      int plo, phi;
      kd_range(parent, t, P, plo, phi);
      const int mid = plo + (phi - plo) / 2;
      const bool far_right = diff < 0.0f;  // the near child was the lower half
      lo = far_right ? mid : plo;
      hi = far_right ? phi : mid;
      node = 2 * parent + (far_right ? 1 : 0);
      depth = t + 1;
      down = true;
    }
    if (!down) break;
  }
  return bpix == 0x7fffffff ? -1 : bpix;
}
