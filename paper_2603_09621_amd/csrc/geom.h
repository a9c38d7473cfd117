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
// it peaks at d_b* clamped to the interval (likewise for the lower end at -d_b*).  The slab misses
// the ellipsoid if the clamped interval is empty.  Bounds are widened by `tol` (world units), which
// covers the hardware reciprocal and square-root approximations used here (these ranges only cull).
//
// SlabAxes holds the slab-independent part for one (a, b) pair, so that several slabs of the same
// pair share it; slab_extent is branch-free and returns whether the slab meets the ellipsoid
// (amin/amax are meaningless otherwise).
struct SlabAxes {
  float isbb, eb, slope, schur, dstar;
};

__device__ __forceinline__ SlabAxes slab_axes(float saa, float sbb, float sab, float c) {
  SlabAxes k;
  k.isbb = __builtin_amdgcn_rcpf(sbb);
  k.eb = c * __builtin_amdgcn_sqrtf(sbb);
  k.slope = sab * k.isbb;
  k.schur = fmaxf(saa - sab * k.slope, 0.f);
  k.dstar = c * sab * __builtin_amdgcn_rsqf(saa);
  return k;
}

__device__ __forceinline__ bool slab_extent(const SlabAxes &k, float ma, float mb, float c, float lo_b, float hi_b,
                                            float tol, float &amin, float &amax) {
  const float ebt = k.eb + tol;
  const float d0 = fmaxf(lo_b - mb, -ebt);
  const float d1 = fminf(hi_b - mb, ebt);
  const float dm = fminf(fmaxf(k.dstar, d0), d1);
  const float dn = fminf(fmaxf(-k.dstar, d0), d1);
  const float c2 = c * c;
  const float hm = __builtin_amdgcn_sqrtf(fmaxf(fmaf(-dm * k.isbb, dm, c2), 0.f) * k.schur);
  const float hn = __builtin_amdgcn_sqrtf(fmaxf(fmaf(-dn * k.isbb, dn, c2), 0.f) * k.schur);
  amax = fmaf(k.slope, dm, ma) + (hm + tol);
  amin = fmaf(k.slope, dn, ma) - (hn + tol);
  return d0 <= d1;
}

__device__ __forceinline__ bool extent_in_slab(float ma, float mb, float saa, float sbb, float sab, float c, float lo_b,
                                               float hi_b, float tol, float &amin, float &amax) {
  const SlabAxes k = slab_axes(saa, sbb, sab, c);
  return slab_extent(k, ma, mb, c, lo_b, hi_b, tol, amin, amax);
}

// World range [lo, hi] -> inclusive voxel index range on an axis of n voxels (origin o, inverse
// spacing ih); empty (il > ih) if the range misses the axis.
__device__ __forceinline__ void world_to_index(float lo, float hi, float o, float ih, int n, int &il, int &ihx) {
  float a = ceilf((lo - o) * ih);
  float b = floorf((hi - o) * ih);
  a = fmaxf(a, 0.f);
  b = fminf(b, (float)(n - 1));
  if (!(a <= b)) {
    il = 1;
    ihx = 0;
    return;
  }
  il = (int)a;
  ihx = (int)b;
}

// Rounding guard for the conservative extents, world units.
__device__ __forceinline__ float extent_tol(float m, float e, float h) { return 4e-3f * h + 8e-6f * (fabsf(m) + e); }

// Voxel centre coordinate along one axis; one fixed formula for every kernel.
__device__ __forceinline__ float centre(float o, float h, int i) { return fmaf(h, (float)i, o); }

// Row coefficients of the exponent (see EvalRec): for the row through (py, pz),
// q(dx) = Q_xx dx^2 + b dx + c.  Every kernel evaluates a pair through row_coeffs + row_q with the
// same operation order, so the forward, the backward and the pair count take the same inclusion
// decision for every pair.
__device__ __forceinline__ void row_coeffs(const EvalRec &R, float py, float pz, float &dy, float &dz, float &b,
                                           float &c) {
  dy = py - R.r0.y;
  dz = pz - R.r0.z;
  b = fmaf(R.r1.y, dy, R.r1.z * dz);
  c = fmaf(fmaf(R.r2.x, dy, R.r2.y * dz), dy, fmaf(R.r2.z * dz, dz, R.r2.w));
}

__device__ __forceinline__ float row_q(float a, float b, float c, float dx) { return fmaf(fmaf(a, dx, b), dx, c); }

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

}  // namespace gs
