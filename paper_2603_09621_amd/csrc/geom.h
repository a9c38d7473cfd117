// Device geometry helpers shared by the binning and rendering kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "gs_internal.h"

namespace gs {

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

// Extent along axis a of the ellipsoid {(d_a, d_b): [d_a d_b] Sigma2^{-1} [d_a d_b]^T <= c^2}
// (the projection of the 3D ellipsoid onto the (a, b) plane has the marginal covariance
// Sigma2 = [[saa, sab], [sab, sbb]]) restricted to the slab b in [lo_b, hi_b] (world units).
// For fixed offset d_b the a-offsets span (sab / sbb) d_b +- sqrt((c^2 - d_b^2 / sbb) (saa - sab^2 / sbb));
// the upper end is concave in d_b with its maximum at d_b* = c sab / sqrt(saa), so over an interval
// it peaks at d_b* clamped to the interval (likewise for the lower end at -d_b*).  Returns false if
// the slab misses the ellipsoid.  Bounds are widened by `tol` (world units).
__device__ __forceinline__ bool extent_in_slab(float ma, float mb, float saa, float sbb, float sab, float c, float lo_b,
                                               float hi_b, float tol, float &amin, float &amax) {
  float eb = c * sqrtf(sbb);
  float d0 = fmaxf(lo_b - mb, -eb - tol);
  float d1 = fminf(hi_b - mb, eb + tol);
  if (d0 > d1) return false;
  float slope = sab / sbb;
  float schur = fmaxf(saa - sab * slope, 0.f);
  float dstar = c * sab / sqrtf(saa);
  float dm = fminf(fmaxf(dstar, d0), d1);
  float dn = fminf(fmaxf(-dstar, d0), d1);
  float c2 = c * c;
  float hm = sqrtf(fmaxf(c2 - dm * dm / sbb, 0.f) * schur);
  float hn = sqrtf(fmaxf(c2 - dn * dn / sbb, 0.f) * schur);
  amax = ma + slope * dm + hm + tol;
  amin = ma + slope * dn - hn - tol;
  return true;
}

// World range [lo, hi] -> inclusive voxel index range on an axis of n voxels (origin o, spacing h).
__device__ __forceinline__ void world_to_index(float lo, float hi, float o, float h, int n, int &il, int &ih) {
  float a = ceilf((lo - o) / h);
  float b = floorf((hi - o) / h);
  a = fmaxf(a, 0.f);
  b = fminf(b, (float)(n - 1));
  if (!(a <= b)) {
    il = 1;
    ih = 0;
    return;
  }
  il = (int)a;
  ih = (int)b;
}

// Rounding guard for the conservative extents, world units.
__device__ __forceinline__ float extent_tol(float m, float e, float h) { return 2e-3f * h + 4e-6f * (fabsf(m) + e); }

// q(p) = delta^T Q delta with Q = -1/2 log2(e) Sigma^{-1}; one fixed evaluation order shared by
// every kernel, so that the forward and the backward take the same inclusion decision per pair.
__device__ __forceinline__ float qform(const EvalRec &R, float px, float py, float pz, float &dx, float &dy,
                                       float &dz) {
  dx = px - R.r0.x;
  dy = py - R.r0.y;
  dz = pz - R.r0.z;
  float tx = fmaf(R.r1.x, dx, fmaf(R.r2.x, dy, R.r2.y * dz));
  float ty = fmaf(R.r1.y, dy, R.r2.z * dz);
  float tz = R.r1.z * dz;
  return fmaf(dx, tx, fmaf(dy, ty, tz * dz));
}

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

}  // namespace gs
