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

// Pixel of the nearest point by float32 squared distance (ties: the lower pixel index), -1 if the
// frame has no point. Depth-first, near child first; a far child is visited unless its split gap
// squared exceeds the best distance so far (equal gaps are visited, for the tie rule).
__device__ __forceinline__ int kd_nearest(const KdArgs& kd, float vx, float vy, float vz) {
  const int P = *kd.count;
  if (P <= 0) return -1;
  struct Entry {
    int lo, hi, node, depth;
    float gap2;
  };
  Entry stack[32];  // at most one pending far child per depth (levels <= 28)
  int sp = 0;
  float best = __builtin_huge_valf();
  int bpix = 0x7fffffff;
  stack[sp++] = Entry{0, P, 1, 0, 0.0f};
  while (sp > 0) {
    const Entry e = stack[--sp];
    if (e.gap2 > best) continue;
    int lo = e.lo, hi = e.hi, node = e.node, depth = e.depth;
    while (depth < kd.levels) {
      const int mid = lo + (hi - lo) / 2;
      const float diff = __fsub_rn((depth & 1) ? vy : vx, kd.split[node]);
      const float g2 = __fmul_rn(diff, diff);
      if (diff < 0.0f) {  // near: the lower half
        if (g2 <= best && mid < hi) stack[sp++] = Entry{mid, hi, 2 * node + 1, depth + 1, g2};
        hi = mid;
        node = 2 * node;
      } else {
        if (g2 <= best && lo < mid) stack[sp++] = Entry{lo, mid, 2 * node, depth + 1, g2};
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
  }
  return bpix == 0x7fffffff ? -1 : bpix;
}
