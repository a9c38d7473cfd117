// Forward and backward rasterizer kernels (§3.2 Eq. (rendering), §3.3).
//
// Forward: one workgroup of 256 threads per 8x8x4 brick, one voxel per lane; each wave owns a 4x4x4
// quarter of the brick.  The brick's Gaussian list is staged through LDS in chunks of 256 records;
// while staging, each Gaussian is tested against the four quarters and every wave compacts the
// indices of the Gaussians that may touch its quarter, so a wave only iterates over those.  Per
// pair: d^2 as a quadratic form, the inclusive cutoff test, one exp2, and the two accumulations
// (numerator S and denominator W).  Voxels sum their Gaussians in ascending index order.
//
// Backward: one wave per brick, one Gaussian per lane.  The brick's per-voxel factors
// c_p = dL/dI(p) / (W(p) + eps) and I(p) are staged in LDS; each lane walks the rows of its
// Gaussian's box inside the brick, restricted per row to the x-interval of the ellipsoid, and
// accumulates the brick-local sums of dL/dw * (1, delta, delta delta^T) and dL/dA.  The 11 sums of
// each (Gaussian, brick) pair are written to the key's pre-sort slot; a second kernel reduces each
// Gaussian's slots in slot order and applies the chain rule (no atomics; deterministic).
#include <hip/hip_runtime.h>

#include "geom.h"
#include "gs_internal.h"

namespace gs {

constexpr int kFwdThreads = 256;
constexpr int kFwdChunk = 256;

// Conservative test of one Gaussian against the four 4x4x4 quarters of an 8x8x4 brick
// (quarter index = sx + 2 sy).  Uses the ellipsoid's x/y extents inside the brick's z-slab and
// inside each half's x- or y-slab.
__device__ __forceinline__ uint32_t quarter_mask(const BrickGrid &bg, const EvalRec &e, const CullRec &c, float cutoff,
                                                 int x0, int y0, int z0) {
  if (c.c1.z == 0.f) return 0u;
  const float mx = e.r0.x, my = e.r0.y, mz = e.r0.z;
  const float sxx = c.c0.x, syy = c.c0.y, szz = c.c0.z, sxy = c.c0.w, sxz = c.c1.x, syz = c.c1.y;
  const float tx = extent_tol(mx, cutoff * sqrtf(sxx), bg.hx), ty = extent_tol(my, cutoff * sqrtf(syy), bg.hy);
  const float Z0 = bg.oz + bg.hz * z0, Z1 = bg.oz + bg.hz * (z0 + 3);
  float xzl, xzh, yzl, yzh;
  if (!extent_in_slab(mx, mz, sxx, szz, sxz, cutoff, Z0, Z1, tx, xzl, xzh)) return 0u;
  if (!extent_in_slab(my, mz, syy, szz, syz, cutoff, Z0, Z1, ty, yzl, yzh)) return 0u;
  float X0[2], X1[2], Y0[2], Y1[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    X0[h] = bg.ox + bg.hx * (x0 + 4 * h);
    X1[h] = bg.ox + bg.hx * (x0 + 4 * h + 3);
    Y0[h] = bg.oy + bg.hy * (y0 + 4 * h);
    Y1[h] = bg.oy + bg.hy * (y0 + 4 * h + 3);
  }
  float xyl[2], xyh[2], yxl[2], yxh[2];
  bool okxy[2], okyx[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    okxy[h] = extent_in_slab(mx, my, sxx, syy, sxy, cutoff, Y0[h], Y1[h], tx, xyl[h], xyh[h]);
    okyx[h] = extent_in_slab(my, mx, syy, sxx, sxy, cutoff, X0[h], X1[h], ty, yxl[h], yxh[h]);
  }
  uint32_t m = 0;
#pragma unroll
  for (int sy = 0; sy < 2; ++sy)
#pragma unroll
    for (int sx = 0; sx < 2; ++sx) {
      if (!okxy[sy] || !okyx[sx]) continue;
      float xl = fmaxf(xzl, xyl[sy]), xh = fminf(xzh, xyh[sy]);
      float yl = fmaxf(yzl, yxl[sx]), yh = fminf(yzh, yxh[sx]);
      if (xl <= X1[sx] && xh >= X0[sx] && yl <= Y1[sy] && yh >= Y0[sy]) m |= 1u << (sx + 2 * sy);
    }
  return m;
}

template <bool COUNT>
__global__ __launch_bounds__(kFwdThreads) void k_fwd(BrickGrid bg, float thr, float cutoff, float eps,
                                                     const EvalRec *__restrict__ er, const CullRec *__restrict__ cr,
                                                     const uint32_t *__restrict__ sorted_gid,
                                                     const uint32_t *__restrict__ brick_off, const DevStatus *st,
                                                     float *__restrict__ I, float *__restrict__ W,
                                                     unsigned long long *__restrict__ pair_count) {
  if (st->overflow) return;
  __shared__ EvalRec srec[kFwdChunk];
  __shared__ uint8_t smask[kFwdChunk];
  __shared__ uint16_t wlist[kFwdThreads / 64][kFwdChunk];
  __shared__ unsigned long long scount[kFwdThreads / 64];

  const int64_t b = blockIdx.x;
  const int kx = (int)(b % bg.nbx), ky = (int)((b / bg.nbx) % bg.nby), kz = (int)(b / ((int64_t)bg.nbx * bg.nby));
  const int x0 = kx * 8, y0 = ky * 8, z0 = kz * 4;
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const int ix = x0 + (w & 1) * 4 + (l & 3);
  const int iy = y0 + (w >> 1) * 4 + ((l >> 2) & 3);
  const int iz = z0 + (l >> 4);
  const float px = bg.ox + bg.hx * ix, py = bg.oy + bg.hy * iy, pz = bg.oz + bg.hz * iz;
  const uint32_t start = brick_off[b], end = brick_off[b + 1];
  const uint64_t lt = lanemask_lt();

  float Wacc = 0.f, Sacc = 0.f;
  uint32_t npairs = 0;
  for (uint32_t c0 = start; c0 < end; c0 += kFwdChunk) {
    const int cnt = (int)min((uint32_t)kFwdChunk, end - c0);
    if (t < cnt) {
      uint32_t gid = sorted_gid[c0 + t];
      EvalRec e = er[gid];
      CullRec c = cr[gid];
      srec[t] = e;
      smask[t] = (uint8_t)quarter_mask(bg, e, c, cutoff, x0, y0, z0);
    }
    __syncthreads();
    int nw = 0;
    for (int j0 = 0; j0 < cnt; j0 += 64) {
      bool has = (j0 + l < cnt) && ((smask[j0 + l] >> w) & 1);
      uint64_t bal = __ballot(has);
      if (has) wlist[w][nw + __popcll(bal & lt)] = (uint16_t)(j0 + l);
      nw += __popcll(bal);
    }
    __syncthreads();
    for (int j = 0; j < nw; ++j) {
      const EvalRec R = srec[wlist[w][j]];
      float dx, dy, dz;
      float q = qform(R, px, py, pz, dx, dy, dz);
      bool in = q >= thr;
      if (COUNT) {
        npairs += in ? 1u : 0u;
      } else {
        float wt = fast_exp2(q + R.r1.w);
        wt = in ? wt : 0.f;
        Wacc += wt;
        Sacc = fmaf(R.r0.w, wt, Sacc);
      }
    }
    __syncthreads();
  }
  const bool inside = ix < bg.nx && iy < bg.ny && iz < bg.nz;
  if (COUNT) {
    unsigned long long v = inside ? npairs : 0u;
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v += __shfl_down(v, d, 64);
    if (l == 0) scount[w] = v;
    __syncthreads();
    if (t == 0) atomicAdd(pair_count, scount[0] + scount[1] + scount[2] + scount[3]);
  } else if (inside) {
    int64_t v = ((int64_t)iz * bg.ny + iy) * bg.nx + ix;
    I[v] = Sacc / (Wacc + eps);
    if (W) W[v] = Wacc;
  }
}

__global__ void k_zero_u64(unsigned long long *p) {
  if (threadIdx.x == 0) *p = 0ull;
}

hipError_t launch_fwd(const BrickGrid &bg, float cutoff, float eps, const void *ws, const WsLayout &L, float *I,
                      float *W, hipStream_t s) {
  const char *b = (const char *)ws;
  const float thr = -kHalfLog2e * cutoff * cutoff;
  prof_begin(s);
  k_fwd<false><<<(unsigned)bg.nbricks, kFwdThreads, 0, s>>>(
      bg, thr, cutoff, eps, (const EvalRec *)(b + L.evalrec), (const CullRec *)(b + L.cullrec),
      (const uint32_t *)(b + L.sorted_gid), (const uint32_t *)(b + L.brick_off), (const DevStatus *)(b + L.status), I,
      W, nullptr);
  prof_end(s, "render_fwd");
  return hipGetLastError();
}

hipError_t launch_count_pairs(const BrickGrid &bg, float cutoff, const void *ws, const WsLayout &L, int64_t *d_count,
                              hipStream_t s) {
  const char *b = (const char *)ws;
  const float thr = -kHalfLog2e * cutoff * cutoff;
  prof_begin(s);
  k_zero_u64<<<1, 64, 0, s>>>((unsigned long long *)d_count);
  k_fwd<true><<<(unsigned)bg.nbricks, kFwdThreads, 0, s>>>(
      bg, thr, cutoff, 0.f, (const EvalRec *)(b + L.evalrec), (const CullRec *)(b + L.cullrec),
      (const uint32_t *)(b + L.sorted_gid), (const uint32_t *)(b + L.brick_off), (const DevStatus *)(b + L.status),
      nullptr, nullptr, (unsigned long long *)d_count);
  prof_end(s, "count_pairs");
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------------
// Backward, brick-local partial sums.  Partial record of one (Gaussian, brick) key, 3 x float4:
//   p0 = (sum c w, sum k, sum k dx, sum k dy), p1 = (sum k dz, sum k dx dx, sum k dy dy, sum k dz dz),
//   p2 = (sum k dx dy, sum k dx dz, sum k dy dz, 0)
// with c = dL/dI / (W + eps), k = c (A - I) w = dL/dw * w.

constexpr int kBwdThreads = 64;

__global__ __launch_bounds__(kBwdThreads) void k_bwd(BrickGrid bg, float thr, float cutoff, float eps,
                                                     const EvalRec *__restrict__ er, const CullRec *__restrict__ cr,
                                                     const uint32_t *__restrict__ sorted_gid,
                                                     const uint32_t *__restrict__ sorted_slot,
                                                     const uint32_t *__restrict__ brick_off, const DevStatus *st,
                                                     const float *__restrict__ Iv, const float *__restrict__ Wv,
                                                     const float *__restrict__ gI, float4 *__restrict__ part) {
  if (st->overflow) return;
  __shared__ float sc[256], sI[256];
  const int64_t b = blockIdx.x;
  const int kx = (int)(b % bg.nbx), ky = (int)((b / bg.nbx) % bg.nby), kz = (int)(b / ((int64_t)bg.nbx * bg.nby));
  const int x0 = kx * 8, y0 = ky * 8, z0 = kz * 4;
  const int t = threadIdx.x;
  const uint32_t start = brick_off[b], end = brick_off[b + 1];
  if (start == end) return;
  for (int v = t; v < 256; v += kBwdThreads) {
    int gx = x0 + (v & 7), gy = y0 + ((v >> 3) & 7), gz = z0 + (v >> 6);
    float c = 0.f, iv = 0.f;
    if (gx < bg.nx && gy < bg.ny && gz < bg.nz) {
      int64_t g = ((int64_t)gz * bg.ny + gy) * bg.nx + gx;
      c = gI[g] / (Wv[g] + eps);
      iv = Iv[g];
    }
    sc[v] = c;
    sI[v] = iv;
  }
  __syncthreads();
  const int xe = min(x0 + 7, bg.nx - 1), ye = min(y0 + 7, bg.ny - 1), ze = min(z0 + 3, bg.nz - 1);
  for (uint32_t c0 = start; c0 < end; c0 += kBwdThreads) {
    const uint32_t k = c0 + t;
    if (k >= end) continue;
    const uint32_t gid = sorted_gid[k];
    const uint32_t slot = sorted_slot[k];
    const EvalRec R = er[gid];
    const CullRec C = cr[gid];
    const float mx = R.r0.x, my = R.r0.y, mz = R.r0.z, A = R.r0.w;
    float ex = cutoff * sqrtf(C.c0.x), ey = cutoff * sqrtf(C.c0.y), ez = cutoff * sqrtf(C.c0.z);
    int xl, xh, yl, yh, zl, zh;
    world_to_index(mx - ex - extent_tol(mx, ex, bg.hx), mx + ex + extent_tol(mx, ex, bg.hx), bg.ox, bg.hx, bg.nx, xl,
                   xh);
    world_to_index(my - ey - extent_tol(my, ey, bg.hy), my + ey + extent_tol(my, ey, bg.hy), bg.oy, bg.hy, bg.ny, yl,
                   yh);
    world_to_index(mz - ez - extent_tol(mz, ez, bg.hz), mz + ez + extent_tol(mz, ez, bg.hz), bg.oz, bg.hz, bg.nz, zl,
                   zh);
    xl = max(xl, x0);
    xh = min(xh, xe);
    yl = max(yl, y0);
    yh = min(yh, ye);
    zl = max(zl, z0);
    zh = min(zh, ze);
    float sA = 0.f, sk = 0.f, skx = 0.f, sky = 0.f, skz = 0.f;
    float mxx = 0.f, myy = 0.f, mzz = 0.f, mxy = 0.f, mxz = 0.f, myz = 0.f;
    const float a = R.r1.x;  // Q_xx < 0
    for (int iz = zl; iz <= zh; ++iz) {
      const float pz = bg.oz + bg.hz * iz;
      for (int iy = yl; iy <= yh; ++iy) {
        const float py = bg.oy + bg.hy * iy;
        // x-interval of q >= thr on this row: a dx^2 + bb dx + cc >= thr
        const float dy = py - my, dz = pz - mz;
        const float bb = fmaf(R.r2.x, dy, R.r2.y * dz);
        const float cc = fmaf(dy, fmaf(R.r1.y, dy, R.r2.z * dz), R.r1.z * dz * dz);
        const float disc = fmaf(bb, bb, -4.f * a * (cc - thr));
        if (disc < 0.f) continue;
        const float sq = sqrtf(disc);
        const float lo = (-bb + sq) / (2.f * a), hi = (-bb - sq) / (2.f * a);
        int xa, xb;
        world_to_index(mx + lo - 0.02f * bg.hx, mx + hi + 0.02f * bg.hx, bg.ox, bg.hx, bg.nx, xa, xb);
        xa = max(xa, xl);
        xb = min(xb, xh);
        for (int ix = xa; ix <= xb; ++ix) {
          const float px = bg.ox + bg.hx * ix;
          float ddx, ddy, ddz;
          const float q = qform(R, px, py, pz, ddx, ddy, ddz);
          if (q >= thr) {
            const int lv = ((iz - z0) * 8 + (iy - y0)) * 8 + (ix - x0);
            const float wt = fast_exp2(q + R.r1.w);
            const float cp = sc[lv];
            const float tt = cp * wt;
            const float kap = cp * (A - sI[lv]) * wt;
            sA += tt;
            sk += kap;
            const float ux = kap * ddx, uy = kap * ddy, uz = kap * ddz;
            skx += ux;
            sky += uy;
            skz += uz;
            mxx = fmaf(ux, ddx, mxx);
            myy = fmaf(uy, ddy, myy);
            mzz = fmaf(uz, ddz, mzz);
            mxy = fmaf(ux, ddy, mxy);
            mxz = fmaf(ux, ddz, mxz);
            myz = fmaf(uy, ddz, myz);
          }
        }
      }
    }
    float4 *o = part + (int64_t)slot * 3;
    o[0] = make_float4(sA, sk, skx, sky);
    o[1] = make_float4(skz, mxx, myy, mzz);
    o[2] = make_float4(mxy, mxz, myz, 0.f);
  }
}

hipError_t launch_bwd(const BrickGrid &bg, float cutoff, float eps, void *ws, const WsLayout &L, const float *I,
                      const float *W, const float *dLdI, hipStream_t s) {
  char *b = (char *)ws;
  const float thr = -kHalfLog2e * cutoff * cutoff;
  prof_begin(s);
  k_bwd<<<(unsigned)bg.nbricks, kBwdThreads, 0, s>>>(
      bg, thr, cutoff, eps, (const EvalRec *)(b + L.evalrec), (const CullRec *)(b + L.cullrec),
      (const uint32_t *)(b + L.sorted_gid), (const uint32_t *)(b + L.sorted_slot), (const uint32_t *)(b + L.brick_off),
      (const DevStatus *)(b + L.status), I, W, dLdI, (float4 *)(b + L.partials));
  prof_end(s, "render_bwd");
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------------
// Per-Gaussian reduction of the brick partials (slot order) and chain rule:
//   dmu = P sum(k delta);  dL/dP = -1/2 sum(k delta delta^T);  dA = sum(c w);  dr = sum(k) / r;
//   P = R D R^T, D = diag(exp(-2 s)):  ds_k = -2 D_k (R^T G R)_kk,  dR = 2 G R D,
//   dqhat from dR through the rotation of a unit quaternion, dq = (dqhat - (qhat.dqhat) qhat) / |q|.

__global__ void k_reduce_chain(int64_t n, const float *__restrict__ quat, const float *__restrict__ ls,
                               const float *__restrict__ relax, const uint32_t *__restrict__ off,
                               const float4 *__restrict__ part, const DevStatus *st, float *__restrict__ d_mu,
                               float *__restrict__ d_ls, float *__restrict__ d_quat, float *__restrict__ d_amp,
                               float *__restrict__ d_relax) {
  if (st->overflow) return;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t s0 = off[i], s1 = off[i + 1];
  float4 a0 = make_float4(0, 0, 0, 0), a1 = a0, a2 = a0;
  for (uint32_t s = s0; s < s1; ++s) {
    const float4 p0 = part[(int64_t)s * 3], p1 = part[(int64_t)s * 3 + 1], p2 = part[(int64_t)s * 3 + 2];
    a0.x += p0.x; a0.y += p0.y; a0.z += p0.z; a0.w += p0.w;
    a1.x += p1.x; a1.y += p1.y; a1.z += p1.z; a1.w += p1.w;
    a2.x += p2.x; a2.y += p2.y; a2.z += p2.z;
  }
  const float sA = a0.x, sk = a0.y;
  const float kd[3] = {a0.z, a0.w, a1.x};
  // G = dL/dP = -1/2 M (symmetric)
  const float G[3][3] = {{-0.5f * a1.y, -0.5f * a2.x, -0.5f * a2.y},
                         {-0.5f * a2.x, -0.5f * a1.z, -0.5f * a2.z},
                         {-0.5f * a2.y, -0.5f * a2.z, -0.5f * a1.w}};
  float qw = quat[4 * i], qx = quat[4 * i + 1], qy = quat[4 * i + 2], qz = quat[4 * i + 3];
  float qn = sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
  if (!(qn > 0.f) || !isfinite(qn)) qn = 1.f;
  const float w = qw / qn, x = qx / qn, y = qy / qn, z = qz / qn;
  const float R[3][3] = {{1.f - 2.f * (y * y + z * z), 2.f * (x * y - w * z), 2.f * (x * z + w * y)},
                         {2.f * (x * y + w * z), 1.f - 2.f * (x * x + z * z), 2.f * (y * z - w * x)},
                         {2.f * (x * z - w * y), 2.f * (y * z + w * x), 1.f - 2.f * (x * x + y * y)}};
  const float D[3] = {expf(-2.f * ls[3 * i]), expf(-2.f * ls[3 * i + 1]), expf(-2.f * ls[3 * i + 2])};
  float P[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) P[r][c] = R[r][0] * D[0] * R[c][0] + R[r][1] * D[1] * R[c][1] + R[r][2] * D[2] * R[c][2];
  if (d_mu) {
#pragma unroll
    for (int r = 0; r < 3; ++r) d_mu[3 * i + r] = P[r][0] * kd[0] + P[r][1] * kd[1] + P[r][2] * kd[2];
  }
  float GR[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) GR[r][c] = G[r][0] * R[0][c] + G[r][1] * R[1][c] + G[r][2] * R[2][c];
  if (d_ls) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      float rtgr = R[0][k] * GR[0][k] + R[1][k] * GR[1][k] + R[2][k] * GR[2][k];
      d_ls[3 * i + k] = -2.f * D[k] * rtgr;
    }
  }
  if (d_quat) {
    float dR[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) dR[r][c] = 2.f * GR[r][c] * D[c];
    float gw = 2.f * (-z * dR[0][1] + y * dR[0][2] + z * dR[1][0] - x * dR[1][2] - y * dR[2][0] + x * dR[2][1]);
    float gx = 2.f * (y * dR[0][1] + z * dR[0][2] + y * dR[1][0] - 2.f * x * dR[1][1] - w * dR[1][2] + z * dR[2][0] +
                      w * dR[2][1] - 2.f * x * dR[2][2]);
    float gy = 2.f * (-2.f * y * dR[0][0] + x * dR[0][1] + w * dR[0][2] + x * dR[1][0] + z * dR[1][2] -
                      w * dR[2][0] + z * dR[2][1] - 2.f * y * dR[2][2]);
    float gz = 2.f * (-2.f * z * dR[0][0] - w * dR[0][1] + x * dR[0][2] + w * dR[1][0] - 2.f * z * dR[1][1] +
                      y * dR[1][2] + x * dR[2][0] + y * dR[2][1]);
    float dot = w * gw + x * gx + y * gy + z * gz;
    d_quat[4 * i] = (gw - dot * w) / qn;
    d_quat[4 * i + 1] = (gx - dot * x) / qn;
    d_quat[4 * i + 2] = (gy - dot * y) / qn;
    d_quat[4 * i + 3] = (gz - dot * z) / qn;
  }
  if (d_amp) d_amp[i] = sA;
  if (d_relax) d_relax[i] = relax ? sk / relax[i] : sk;
}

hipError_t launch_reduce_chain(const gs_gaussians_t &g, const void *ws, const WsLayout &L, const gs_grads_t &gr,
                               hipStream_t s) {
  if (g.n == 0) return hipSuccess;
  const char *b = (const char *)ws;
  prof_begin(s);
  k_reduce_chain<<<(unsigned)((g.n + 255) / 256), 256, 0, s>>>(
      g.n, g.quat, g.log_scale, g.relax, (const uint32_t *)(b + L.off), (const float4 *)(b + L.partials),
      (const DevStatus *)(b + L.status), gr.d_mu, gr.d_log_scale, gr.d_quat, gr.d_amp,
      g.relax ? gr.d_relax : nullptr);
  prof_end(s, "reduce_chain");
  return hipGetLastError();
}

}  // namespace gs
