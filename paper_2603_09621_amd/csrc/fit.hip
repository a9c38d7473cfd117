// Losses of the per-scan fit and the Adam update (elementwise, HBM-bound).
//
// Loss values are reduced deterministically: per-block partial sums in a fixed order, then one
// block sums the partials in a fixed order.
#include <hip/hip_runtime.h>

#include <cmath>

#include "geom.h"
#include "gs_internal.h"

namespace gs {

int loss_blocks(int64_t nvox) {
  int64_t per = (int64_t)kLossThreads * kLossItems;
  return (int)((nvox + per - 1) / per);
}

__device__ __forceinline__ float block_sum(float v, float *sh) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_down(v, d, 64);
  if (lane_id() == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  float s = 0.f;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
  return s;
}

__global__ __launch_bounds__(kLossThreads) void k_loss_mse(const float *__restrict__ I, const float *__restrict__ T,
                                                            int64_t n, float scale, float *__restrict__ g,
                                                            float *__restrict__ partial) {
  __shared__ float sh[kLossThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kLossThreads * kLossItems;
  float acc = 0.f;
#pragma unroll 4
  for (int j = 0; j < kLossItems; ++j) {
    int64_t v = base + (int64_t)j * kLossThreads + threadIdx.x;
    if (v < n) {
      float d = I[v] - T[v];
      g[v] = scale * d;
      acc = fmaf(d, d, acc);
    }
  }
  float s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// LR voxel q = (k, y, x): lr = (((I[fk] + I[fk+1]) + ...) + I[fk+f-1]) * (1/f); diff = lr - obs;
// dL/dI = sign(diff) * gscale on the f HR voxels of q.  st (a fit step's binning status, or NULL):
// after a key-capacity overflow the step writes nothing, this kernel included.
__global__ __launch_bounds__(kLossThreads) void k_loss_l1z(const float *__restrict__ I, const float *__restrict__ obs,
                                                            int64_t nlr, int64_t plane, int f, float invf, float gscale,
                                                            float *__restrict__ g, float *__restrict__ partial,
                                                            const DevStatus *st) {
  if (st && st->overflow) return;
  __shared__ float sh[kLossThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kLossThreads * kLossItems;
  float acc = 0.f;
  for (int j = 0; j < kLossItems; ++j) {
    int64_t q = base + (int64_t)j * kLossThreads + threadIdx.x;
    if (q < nlr) {
      int64_t k = q / plane, r = q - k * plane;
      int64_t h0 = k * f * plane + r;
      float s = I[h0];
      for (int z = 1; z < f; ++z) s = s + I[h0 + z * plane];
      float lr = s * invf;
      float d = lr - obs[q];
      float sg = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
      for (int z = 0; z < f; ++z) g[h0 + z * plane] = sg * gscale;
      acc += fabsf(d);
    }
  }
  float s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_loss_finalize(const float *__restrict__ partial, int nb, float scale,
                                                       float *__restrict__ loss, const DevStatus *st = nullptr) {
  if (st && st->overflow) return;
  __shared__ float sh[4];
  float acc = 0.f;
  for (int i = threadIdx.x; i < nb; i += 256) acc += partial[i];
  float s = block_sum(acc, sh);
  if (threadIdx.x == 0) *loss = s * scale;
}

hipError_t launch_loss_mse(const float *I, const float *T, int64_t nvox, float *g, float *loss, void *scratch,
                           hipStream_t s) {
  int nb = loss_blocks(nvox);
  if (nb == 0) return hipSuccess;
  prof_begin(s);
  k_loss_mse<<<nb, kLossThreads, 0, s>>>(I, T, nvox, (float)(2.0 / (double)nvox), g, (float *)scratch);
  k_loss_finalize<<<1, 256, 0, s>>>((const float *)scratch, nb, (float)(1.0 / (double)nvox), loss);
  prof_end(s, "loss_mse");
  return hipGetLastError();
}

hipError_t launch_loss_l1z(const float *I, const float *obs, int nx, int ny, int nz, int f, float *g, float *loss,
                           void *scratch, hipStream_t s, const DevStatus *st) {
  int64_t plane = (int64_t)nx * ny;
  int64_t nlr = plane * (nz / f);
  int nb = loss_blocks(nlr);
  if (nb == 0) return hipSuccess;
  prof_begin(s);
  k_loss_l1z<<<nb, kLossThreads, 0, s>>>(I, obs, nlr, plane, f, (float)(1.0 / f), (float)(1.0 / ((double)f * nlr)),
                                         g, (float *)scratch, st);
  k_loss_finalize<<<1, 256, 0, s>>>((const float *)scratch, nb, (float)(1.0 / (double)nlr), loss, st);
  prof_end(s, "loss_l1z");
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------------
// Adam with bias correction over the parameter groups mu (3n), log_scale (3n), quat (4n), amp (n),
// relax (n, optional).  The step counter lives on the device: this step is *step + 1.

struct AdamGroups {
  float *p[5];
  const float *g[5];
  float lr[5];
  int64_t end[5];  // cumulative element counts
};

__global__ void k_adam(AdamGroups G, int ngroups, int64_t total, float *__restrict__ m, float *__restrict__ v, float b1,
                       float b2, float eps, float lnb1, float lnb2, const int32_t *__restrict__ step,
                       const DevStatus *st) {
  if (st && st->overflow) return;
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  int gi = 0;
  while (gi < ngroups - 1 && e >= G.end[gi]) ++gi;
  const int64_t j = e - (gi ? G.end[gi - 1] : 0);
  const float t = (float)(*step + 1);
  const float bc1 = -expm1f(t * lnb1), bc2 = -expm1f(t * lnb2);
  const float g = G.g[gi][j];
  const float mm = fmaf(b1, m[e], (1.f - b1) * g);
  const float vv = fmaf(b2, v[e], (1.f - b2) * g * g);
  m[e] = mm;
  v[e] = vv;
  const float lr = G.lr[gi];
  if (lr != 0.f) G.p[gi][j] -= lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
}

__global__ void k_step_inc(int32_t *step, const DevStatus *st) {
  if (threadIdx.x == 0 && !(st && st->overflow)) *step += 1;
}

hipError_t launch_adam(const gs_fit_state_t &st, const gs_grads_t &gr, const gs_adam_t &hp, const void *ws_status,
                       hipStream_t s) {
  const int64_t n = st.n;
  if (n == 0) return hipSuccess;
  AdamGroups G;
  float *ps[5] = {st.mu, st.log_scale, st.quat, st.amp, st.relax};
  const float *gs_[5] = {gr.d_mu, gr.d_log_scale, gr.d_quat, gr.d_amp, gr.d_relax};
  const int64_t sz[5] = {3 * n, 3 * n, 4 * n, n, n};
  int ng = st.relax ? 5 : 4;
  int64_t acc = 0;
  for (int k = 0; k < 5; ++k) {
    G.p[k] = ps[k];
    G.g[k] = gs_[k];
    G.lr[k] = hp.lr[k];
    acc += (k < ng) ? sz[k] : 0;
    G.end[k] = acc;
  }
  // the moment arrays keep the fixed 12n layout: relax moments (if any) start at 11n
  const DevStatus *dst = (const DevStatus *)ws_status;
  prof_begin(s);
  k_adam<<<(unsigned)((acc + 255) / 256), 256, 0, s>>>(G, ng, acc, st.m, st.v, hp.beta1, hp.beta2, hp.eps,
                                                       (float)std::log((double)hp.beta1),
                                                       (float)std::log((double)hp.beta2), st.step, dst);
  k_step_inc<<<1, 64, 0, s>>>(st.step, dst);
  prof_end(s, "adam");
  return hipGetLastError();
}

}  // namespace gs
