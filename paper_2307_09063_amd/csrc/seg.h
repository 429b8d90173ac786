// Launches over a list of segments (each segment a group of clips of one map size, with its own
// batch-norm statistics).  One grid carries the workgroups of every segment back to back:
// segment s owns workgroups base[s] .. base[s] + grid[s] - 1, where it runs as workgroups
// 0 .. grid[s] - 1 of a grid of grid[s] with its own arguments a[s].  So one launch per kernel
// kind walks the tile lists of all segments, and a kernel body is the same code for one segment
// or many.  Every segment starts at a multiple of 8 workgroups (a few slots before it may stay
// idle and exit at once), so that the XCD-aware schedules, which read the XCD from the low three
// bits of the workgroup index, see the hardware's XCD numbering in every segment.
#pragma once
#include <hip/hip_runtime.h>

#include "plan.h"

namespace stda {

template <class A>
struct SegL {
  int n;
  int base[kMaxSegs];
  int grid[kMaxSegs];
  A a[kMaxSegs];
};

struct SegB {
  int s, x, gx;  // segment, workgroup index inside it, its workgroup count
};

template <class A>
__device__ __forceinline__ SegB seg_block(const SegL<A>& L) {
  int s = 0;
  while (s + 1 < L.n && (int)blockIdx.x >= L.base[s + 1]) ++s;
  return SegB{s, (int)blockIdx.x - L.base[s], L.grid[s]};
}

}  // namespace stda
