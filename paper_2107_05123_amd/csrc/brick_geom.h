// Brick-local geometry shared by the host builder and the device kernels.
//
// A brick holds B^d leaves; its (B+1)^d node positions are numbered
// lexicographically (x fastest, the marching axis last).  Positions on the
// brick boundary get a compact rank in that order; a brick's boundary partial
// sums live at slot_base + brick * n_boundary + rank.
#pragma once
#include <hip/hip_runtime.h>

namespace chns {

__host__ __device__ inline int brick_boundary_count(int dim, int B) {
  const int n1 = B + 1;
  if (dim == 3) return n1 * n1 * n1 - (B - 1) * (B - 1) * (B - 1) * (B > 1);
  return n1 * n1 - (B - 1) * (B - 1) * (B > 1);
}

// Rank of boundary position (jx, jy, z) in 3D (jy unused in 2D, where the
// layer is the row of B+1 nodes at height z).  Undefined for interior ones.
__host__ __device__ inline int brick_rank(int dim, int B, int jx, int jy, int z) {
  const int n1 = B + 1;
  if (dim == 2) {
    if (z == 0) return jx;
    const int r = n1 + (z - 1) * 2;
    if (z == B) return r + jx;
    return r + (jx == 0 ? 0 : 1);
  }
  const int full = n1 * n1;
  const int ring = full - (B - 1) * (B - 1);
  if (z == 0) return jx + n1 * jy;
  int r = full + (z - 1) * ring;
  if (z == B) return r + jx + n1 * jy;
  if (jy == 0) return r + jx;
  r += n1 + (jy - 1) * 2;
  if (jy == B) return r + jx;
  return r + (jx == 0 ? 0 : 1);
}

}  // namespace chns
