// Per-Gaussian reduction of the backward's brick partials and the chain rule (§3.3 gradient
// equations; the parameterisation of §3.1), optionally fused with the Adam update of the fit step.
#include <hip/hip_runtime.h>

#include <cmath>

#include "geom.h"
#include "gs_internal.h"

namespace gs {

// ------------------------------------------------------------------------------------------------
// Per-Gaussian reduction of the brick partials (slot order) and chain rule:
//   dmu = P sum(k delta);  dL/dP = -1/2 sum(k delta delta^T);  dA = sum(c w);  dr = sum(k) / r;
//   P = R D R^T, D = diag(exp(-2 s)):  ds_k = -2 D_k (R^T G R)_kk,  dR = 2 G R D,
//   dqhat from dR through the rotation of a unit quaternion, dq = (dqhat - (qhat.dqhat) qhat) / |q|.

// Per-Gaussian sums of the brick partials, for the 256 consecutive Gaussians of a block: the
// block's partials (contiguous, since keys are numbered Gaussian-major) are loaded cooperatively
// through LDS in chunks, and each thread adds its own Gaussian's partials in slot order (a Gaussian
// with more than kLongKeys partials is left to block_long_sums, so that one long list does not
// hold the block).  The next
// chunk's loads are issued into registers before the current chunk is summed.
constexpr int kRedThreads = 256;
constexpr int kRedChunk = 768;                         // partials per LDS chunk (36 KB)
constexpr int kRedPer = 3 * kRedChunk / kRedThreads;  // float4 loads per thread per chunk

// A Gaussian with more partials than this is summed by a wave (block_long_sums) instead of its
// own thread.
constexpr uint32_t kLongKeys = 64;

__device__ __forceinline__ void block_partial_sums(int64_t i0, int64_t n, const uint32_t *__restrict__ off,
                                                   const float4 *__restrict__ part, float4 *sp, float4 &a0,
                                                   float4 &a1, float4 &a2, uint32_t &count) {
  const int t = threadIdx.x;
  const int64_t i = i0 + t;
  const int64_t iend = min(i0 + (int64_t)kRedThreads, n);
  const uint32_t sb = off[i0], se = off[iend];
  uint32_t my0 = i < n ? off[i] : se, my1 = i < n ? off[i + 1] : se;
  count = my1 - my0;
  if (count > kLongKeys) my1 = my0;  // summed by block_long_sums
  a0 = make_float4(0, 0, 0, 0);
  a1 = a0;
  a2 = a0;
  float4 r[kRedPer];
  if (sb < se) {
    const int m3 = 3 * (int)min((uint32_t)kRedChunk, se - sb);
#pragma unroll
    for (int j = 0; j < kRedPer; ++j) {
      const int k = t + j * kRedThreads;
      r[j] = k < m3 ? part[(int64_t)sb * 3 + k] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
  for (uint32_t c0 = sb; c0 < se; c0 += kRedChunk) {
    const int m = (int)min((uint32_t)kRedChunk, se - c0);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kRedPer; ++j) sp[t + j * kRedThreads] = r[j];
    __syncthreads();
    const uint32_t c1 = c0 + kRedChunk;
    if (c1 < se) {
      const int m3 = 3 * (int)min((uint32_t)kRedChunk, se - c1);
#pragma unroll
      for (int j = 0; j < kRedPer; ++j) {
        const int k = t + j * kRedThreads;
        r[j] = k < m3 ? part[(int64_t)c1 * 3 + k] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
    const uint32_t lo = max(my0, c0), hi = min(my1, c0 + (uint32_t)m);
    for (uint32_t s = lo; s < hi; ++s) {
      const int q = (int)(s - c0) * 3;
      const float4 p0 = sp[q], p1 = sp[q + 1], p2 = sp[q + 2];
      a0.x += p0.x; a0.y += p0.y; a0.z += p0.z; a0.w += p0.w;
      a1.x += p1.x; a1.y += p1.y; a1.z += p1.z; a1.w += p1.w;
      a2.x += p2.x; a2.y += p2.y; a2.z += p2.z;
    }
  }
}

// Sums of the long partial lists of a block's Gaussians: each wave takes the block's long Gaussians
// in turn (w, w + 4, ... of them in index order); lane l adds the Gaussian's partials l, l + 64, ...
// in order, and a fixed butterfly adds the 64 lane sums.  The order depends only on the Gaussian's own
// partials, so the result is the same whatever block or batch the Gaussian falls in.  The owner
// thread's (a0, a1, a2) receive the sums.
__device__ __forceinline__ float bfly_sum(float v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

__device__ __forceinline__ void block_long_sums(int64_t i0, const uint32_t *__restrict__ off,
                                                const float4 *__restrict__ part, float4 *sp, uint32_t c,
                                                float4 &a0, float4 &a1, float4 &a2) {
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  // (a barrier: the partial sums' use of sp is over)
  if (!__syncthreads_or(c > kLongKeys ? 1 : 0)) return;  // no long list in the block
  __shared__ uint64_t slong[kRedThreads / 64];
  const uint64_t m = __ballot(c > kLongKeys);
  if (l == 0) slong[w] = m;
  __syncthreads();
  int k = 0;  // running index over the block's long Gaussians
  for (int ww = 0; ww < kRedThreads / 64; ++ww) {
    for (uint64_t mm = slong[ww]; mm; mm &= mm - 1, ++k) {
      if ((k & (kRedThreads / 64 - 1)) != w) continue;  // uniform per wave
      const int src = ww * 64 + __ffsll((unsigned long long)mm) - 1;
      const uint32_t s0 = off[i0 + src], s1 = off[i0 + src + 1];
      float v[11] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      for (uint32_t s = s0 + (uint32_t)l; s < s1; s += 64) {
        const float4 p0 = part[(int64_t)s * 3], p1 = part[(int64_t)s * 3 + 1], p2 = part[(int64_t)s * 3 + 2];
        v[0] += p0.x; v[1] += p0.y; v[2] += p0.z; v[3] += p0.w;
        v[4] += p1.x; v[5] += p1.y; v[6] += p1.z; v[7] += p1.w;
        v[8] += p2.x; v[9] += p2.y; v[10] += p2.z;
      }
#pragma unroll
      for (int q = 0; q < 11; ++q) v[q] = bfly_sum(v[q]);
      // hand the sums to the owner thread through LDS (it may sit in another wave)
      if (l == 0) {
        sp[3 * src] = make_float4(v[0], v[1], v[2], v[3]);
        sp[3 * src + 1] = make_float4(v[4], v[5], v[6], v[7]);
        sp[3 * src + 2] = make_float4(v[8], v[9], v[10], 0.f);
      }
    }
  }
  __syncthreads();
  if (c > kLongKeys) {
    a0 = sp[3 * t];
    a1 = sp[3 * t + 1];
    a2 = sp[3 * t + 2];
  }
}

// Gradient of Gaussian i from its summed partials (a0, a1, a2) and its raw parameters.
// g[0..2] = dmu, g[3..5] = dlog_scale, g[6..9] = dquat, g[10] = dA, g[11] = dr (r = 1 if relax NULL).
__device__ __forceinline__ void gauss_grad_v(float qw, float qx, float qy, float qz, float s0, float s1, float s2,
                                             float r, float4 a0, float4 a1, float4 a2, float g[12]) {
  const float sA = a0.x, sk = a0.y;
  const float kd[3] = {a0.z, a0.w, a1.x};
  // G = dL/dP = -1/2 M (symmetric)
  const float G[3][3] = {{-0.5f * a1.y, -0.5f * a2.x, -0.5f * a2.y},
                         {-0.5f * a2.x, -0.5f * a1.z, -0.5f * a2.z},
                         {-0.5f * a2.y, -0.5f * a2.z, -0.5f * a1.w}};
  float qn = sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
  if (!(qn > 0.f) || !isfinite(qn)) qn = 1.f;
  const float w = qw / qn, x = qx / qn, y = qy / qn, z = qz / qn;
  const float R[3][3] = {{1.f - 2.f * (y * y + z * z), 2.f * (x * y - w * z), 2.f * (x * z + w * y)},
                         {2.f * (x * y + w * z), 1.f - 2.f * (x * x + z * z), 2.f * (y * z - w * x)},
                         {2.f * (x * z - w * y), 2.f * (y * z + w * x), 1.f - 2.f * (x * x + y * y)}};
  const float D[3] = {expf(-2.f * s0), expf(-2.f * s1), expf(-2.f * s2)};
  float P[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) P[r][c] = R[r][0] * D[0] * R[c][0] + R[r][1] * D[1] * R[c][1] + R[r][2] * D[2] * R[c][2];
#pragma unroll
  for (int r = 0; r < 3; ++r) g[r] = P[r][0] * kd[0] + P[r][1] * kd[1] + P[r][2] * kd[2];
  float GR[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) GR[r][c] = G[r][0] * R[0][c] + G[r][1] * R[1][c] + G[r][2] * R[2][c];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float rtgr = R[0][k] * GR[0][k] + R[1][k] * GR[1][k] + R[2][k] * GR[2][k];
    g[3 + k] = -2.f * D[k] * rtgr;
  }
  float dR[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) dR[r][c] = 2.f * GR[r][c] * D[c];
  const float gw = 2.f * (-z * dR[0][1] + y * dR[0][2] + z * dR[1][0] - x * dR[1][2] - y * dR[2][0] + x * dR[2][1]);
  const float gx = 2.f * (y * dR[0][1] + z * dR[0][2] + y * dR[1][0] - 2.f * x * dR[1][1] - w * dR[1][2] +
                          z * dR[2][0] + w * dR[2][1] - 2.f * x * dR[2][2]);
  const float gy = 2.f * (-2.f * y * dR[0][0] + x * dR[0][1] + w * dR[0][2] + x * dR[1][0] + z * dR[1][2] -
                          w * dR[2][0] + z * dR[2][1] - 2.f * y * dR[2][2]);
  const float gz = 2.f * (-2.f * z * dR[0][0] - w * dR[0][1] + x * dR[0][2] + w * dR[1][0] - 2.f * z * dR[1][1] +
                          y * dR[1][2] + x * dR[2][0] + y * dR[2][1]);
  const float dot = w * gw + x * gx + y * gy + z * gz;
  g[6] = (gw - dot * w) / qn;
  g[7] = (gx - dot * x) / qn;
  g[8] = (gy - dot * y) / qn;
  g[9] = (gz - dot * z) / qn;
  g[10] = sA;
  g[11] = sk / r;
}

// Gradient of Gaussian i from its summed partials and its raw parameters in global memory
// (r = 1 when relax is NULL).
__device__ __forceinline__ void gauss_grad(int64_t i, const float *__restrict__ quat, const float *__restrict__ ls,
                                           const float *__restrict__ relax, float4 a0, float4 a1, float4 a2,
                                           float g[12]) {
  gauss_grad_v(quat[4 * i], quat[4 * i + 1], quat[4 * i + 2], quat[4 * i + 3], ls[3 * i], ls[3 * i + 1],
               ls[3 * i + 2], relax ? relax[i] : 1.f, a0, a1, a2, g);
}

__global__ void k_reduce_chain(int64_t n, const float *__restrict__ quat, const float *__restrict__ ls,
                               const float *__restrict__ relax, const uint32_t *__restrict__ off,
                               const float4 *__restrict__ part, const DevStatus *st, float *__restrict__ d_mu,
                               float *__restrict__ d_ls, float *__restrict__ d_quat, float *__restrict__ d_amp,
                               float *__restrict__ d_relax) {
  if (st->overflow) return;
  __shared__ float4 sp[3 * kRedChunk];
  const int64_t i0 = (int64_t)blockIdx.x * kRedThreads, i = i0 + threadIdx.x;
  float4 a0, a1, a2;
  uint32_t cnt;
  block_partial_sums(i0, n, off, part, sp, a0, a1, a2, cnt);
  block_long_sums(i0, off, part, sp, cnt, a0, a1, a2);
  if (i >= n) return;
  float g[12];
  gauss_grad(i, quat, ls, relax, a0, a1, a2, g);
  if (d_mu) {
    d_mu[3 * i] = g[0];
    d_mu[3 * i + 1] = g[1];
    d_mu[3 * i + 2] = g[2];
  }
  if (d_ls) {
    d_ls[3 * i] = g[3];
    d_ls[3 * i + 1] = g[4];
    d_ls[3 * i + 2] = g[5];
  }
  if (d_quat) {
    d_quat[4 * i] = g[6];
    d_quat[4 * i + 1] = g[7];
    d_quat[4 * i + 2] = g[8];
    d_quat[4 * i + 3] = g[9];
  }
  if (d_amp) d_amp[i] = g[10];
  if (d_relax) d_relax[i] = g[11];
}

// Fused gradient + Adam for the fit step: the gradient of Gaussian i (as k_reduce_chain, also
// written to the gradient outputs) and the bias-corrected Adam update of its 12 parameters, moments
// in the group layout mu (3n), log_scale (3n), quat (4n), amp (n), relax (n).  Each scan of the table
// has its own step counter, already advanced by this step's binning (the count scan): Gaussian i of
// scan k takes step t = step[k].  Block 0 also writes the fit loss of every scan.
struct AdamArgs {
  float lr[5];
  float b1, b2, eps;
  float lnb1, lnb2;  // ln of the betas: the bias corrections are 1 - beta^t = -expm1(t ln beta)
};

__device__ __forceinline__ void adam_one(float &p, float g, float &m, float &v, float lr, float b1, float b2, float eps,
                                         float bc1, float bc2) {
  const float mm = fmaf(b1, m, (1.f - b1) * g);
  const float vv = fmaf(b2, v, (1.f - b2) * g * g);
  m = mm;
  v = vv;
  if (lr != 0.f) p -= lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
}

// Fit loss of every scan of T: loss[s] = (sum of its bricks' loss parts, fixed order) * lscale, by
// one block of kRedThreads threads.
__device__ void fit_loss_sum(const ScanTable &T, const float *__restrict__ loss_part, float *__restrict__ loss) {
  __shared__ float sh[kRedThreads / 64];
  const int t = threadIdx.x;
  for (int k = 0; k < T.ns; ++k) {
    const ScanDesc &sd = T.s[k];
    const float *lp = loss_part + sd.b0;
    const int64_t nb = sd.bg.nbricks;
    float acc = 0.f;
    for (int64_t j0 = t; j0 < nb; j0 += 8 * kRedThreads) {
      float w8[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int64_t jj = j0 + (int64_t)j * kRedThreads;
        w8[j] = jj < nb ? lp[jj] : 0.f;
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) acc += w8[j];
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) acc += __shfl_down(acc, d, 64);
    if ((t & 63) == 0) sh[t >> 6] = acc;
    __syncthreads();
    if (t == 0) {
      float tot = 0.f;
      for (int w = 0; w < kRedThreads / 64; ++w) tot += sh[w];
      loss[k] = tot * sd.lscale;
    }
    __syncthreads();
  }
}

__global__ void k_reduce_adam(const ScanTable T, int64_t n, float *__restrict__ mu, float *__restrict__ ls, float *__restrict__ quat,
                              float *__restrict__ amp, float *__restrict__ relax, const uint32_t *__restrict__ off,
                              const float4 *__restrict__ part, const DevStatus *st, float *__restrict__ d_mu,
                              float *__restrict__ d_ls, float *__restrict__ d_quat, float *__restrict__ d_amp,
                              float *__restrict__ d_relax, float *__restrict__ m, float *__restrict__ v,
                              const int32_t *__restrict__ step, AdamArgs h, const float *__restrict__ loss_part,
                              float *__restrict__ loss) {
  if (st->overflow) return;
  // block 0 also sums the fit loss of every scan (the per-brick loss parts come from the backward):
  // bricks t, t + 256, ... per thread in order, then a fixed-order block reduction
  if (blockIdx.x == 0 && loss_part) fit_loss_sum(T, loss_part, loss);
  __shared__ float4 sp[3 * kRedChunk];
  const int64_t i0 = (int64_t)blockIdx.x * kRedThreads, i = i0 + threadIdx.x;
  // the Gaussian's parameters and moments do not depend on the partial sums: their loads are issued
  // first, so that they overlap the partials' loads.  Entry e of the 12 is (group, component) in the
  // order mu 3, log_scale 3, quat 4, amp, relax; its moment index is moff[e] (group layout).
  const int ng = relax ? 12 : 11;
  auto moff = [&](int e) -> int64_t {
    return e < 3 ? 3 * i + e : e < 6 ? 3 * n + 3 * i + (e - 3) : e < 10 ? 6 * n + 4 * i + (e - 6)
                                                                     : (e == 10 ? 10 * n + i : 11 * n + i);
  };
  float pv[12], mv[12], vv[12];
#pragma unroll
  for (int e = 0; e < 12; ++e) {
    pv[e] = 1.f;
    mv[e] = 0.f;
    vv[e] = 0.f;
  }
  if (i < n) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      pv[a] = mu[3 * i + a];
      pv[3 + a] = ls[3 * i + a];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) pv[6 + a] = quat[4 * i + a];
    pv[10] = amp[i];
    if (relax) pv[11] = relax[i];
#pragma unroll
    for (int e = 0; e < 12; ++e)
      if (e < ng) {
        mv[e] = m[moff(e)];
        vv[e] = v[moff(e)];
      }
  }
  float4 a0, a1, a2;
  uint32_t cnt;
  block_partial_sums(i0, n, off, part, sp, a0, a1, a2, cnt);
  block_long_sums(i0, off, part, sp, cnt, a0, a1, a2);
  if (i >= n) return;
  float g[12];
  gauss_grad_v(pv[6], pv[7], pv[8], pv[9], pv[3], pv[4], pv[5], pv[11], a0, a1, a2, g);
  const float t = (float)step[T.of_gauss(i)];  // advanced by this step's binning
  const float bc1 = -expm1f(t * h.lnb1), bc2 = -expm1f(t * h.lnb2);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    d_mu[3 * i + a] = g[a];
    d_ls[3 * i + a] = g[3 + a];
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) d_quat[4 * i + a] = g[6 + a];
  d_amp[i] = g[10];
  if (relax && d_relax) d_relax[i] = g[11];
#pragma unroll
  for (int e = 0; e < 12; ++e) {
    if (e >= ng) continue;
    const int grp = e < 3 ? 0 : e < 6 ? 1 : e < 10 ? 2 : e == 10 ? 3 : 4;
    adam_one(pv[e], g[e], mv[e], vv[e], h.lr[grp], h.b1, h.b2, h.eps, bc1, bc2);
    m[moff(e)] = mv[e];
    v[moff(e)] = vv[e];
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    mu[3 * i + a] = pv[a];
    ls[3 * i + a] = pv[3 + a];
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) quat[4 * i + a] = pv[6 + a];
  amp[i] = pv[10];
  if (relax) relax[i] = pv[11];
}

// Fit loss without Gaussians (the fused reduction computes it otherwise), one block per scan:
// loss[s] = (sum of the scan's per-brick loss parts, fixed order) * lscale.  Thread t adds bricks
// t, t + 1024, ... in order, 8 loads in flight.
constexpr int kFinThreads = 1024;

__global__ __launch_bounds__(kFinThreads) void k_fit_finalize(const ScanTable T, const float *__restrict__ loss_part,
                                                              float *__restrict__ loss, const DevStatus *st) {
  __shared__ float sh[kFinThreads / 64];
  const ScanDesc &sd = T.s[blockIdx.x];
  float acc = 0.f;
  const float *lp = loss_part + sd.b0;
  const int64_t nb = sd.bg.nbricks;
  for (int64_t i0 = threadIdx.x; i0 < nb; i0 += 8 * kFinThreads) {
    float v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int64_t i = i0 + (int64_t)j * kFinThreads;
      v[j] = i < nb ? lp[i] : 0.f;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) acc += v[j];
  }
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) acc += __shfl_down(acc, d, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0 && !st->overflow) {
    float tot = 0.f;
    for (int w = 0; w < kFinThreads / 64; ++w) tot += sh[w];
    loss[blockIdx.x] = tot * sd.lscale;
  }
}

hipError_t launch_reduce_adam(const ScanTable &T, const gs_fit_state_t &g, const void *ws, const WsLayout &L,
                              const gs_grads_t &gr, const gs_adam_t &hp, const float *loss_part, float *loss,
                              hipStream_t s) {
  const char *b = (const char *)ws;
  AdamArgs h;
  for (int k = 0; k < 5; ++k) h.lr[k] = hp.lr[k];
  h.b1 = hp.beta1;
  h.b2 = hp.beta2;
  h.eps = hp.eps;
  h.lnb1 = (float)std::log((double)hp.beta1);
  h.lnb2 = (float)std::log((double)hp.beta2);
  prof_begin(s);
  if (g.n > 0)
    k_reduce_adam<<<(unsigned)((g.n + kRedThreads - 1) / kRedThreads), kRedThreads, 0, s>>>(
        T, g.n, g.mu, g.log_scale, g.quat, g.amp, g.relax, (const uint32_t *)(b + L.off),
        (const float4 *)(b + L.partials), (const DevStatus *)(b + L.status), gr.d_mu, gr.d_log_scale, gr.d_quat,
        gr.d_amp, gr.d_relax, g.m, g.v, g.step, h, loss_part, loss);
  else if (loss_part)
    k_fit_finalize<<<(unsigned)T.ns, kFinThreads, 0, s>>>(T, loss_part, loss, (const DevStatus *)(b + L.status));
  prof_end(s, "reduce_adam");
  return hipGetLastError();
}

hipError_t launch_reduce_chain(const gs_gaussians_t &g, const void *ws, const WsLayout &L, const gs_grads_t &gr,
                               hipStream_t s) {
  if (g.n == 0) return hipSuccess;
  const char *b = (const char *)ws;
  prof_begin(s);
  k_reduce_chain<<<(unsigned)((g.n + kRedThreads - 1) / kRedThreads), kRedThreads, 0, s>>>(
      g.n, g.quat, g.log_scale, g.relax, (const uint32_t *)(b + L.off), (const float4 *)(b + L.partials),
      (const DevStatus *)(b + L.status), gr.d_mu, gr.d_log_scale, gr.d_quat, gr.d_amp,
      g.relax ? gr.d_relax : nullptr);
  prof_end(s, "reduce_chain");
  return hipGetLastError();
}

}  // namespace gs
