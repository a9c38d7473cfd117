// Forward and backward rasterizer kernels (§3.2 Eq. (rendering), §3.3).
//
// Bricks are BX x 8 x 4 voxels (BX in {4, 8, 16}; the paper uses 8 x 8 x 4).  Every launch covers
// the bricks of all scans of a scan table (the forward: one workgroup per brick; the backward: one
// per group of G consecutive bricks of a scan).
//
// Forward: BX/2 waves per brick; each wave owns a 4x4x4 quarter of the brick, split into four
// 4x2x2 cells.  The brick's Gaussian list is staged through LDS in chunks; while staging, each
// Gaussian is tested against every cell and each wave compacts, per cell of its quarter, the
// Gaussians that may touch the cell.  A 16-lane group works on one cell and keeps four Gaussians in
// flight: lanes 4j..4j+3 of the group take entries j, j+4, j+8, ... of the cell's list; each lane owns
// one voxel row of 4 voxels along x, sets up the row's quadratic once per Gaussian and evaluates the
// 4 voxels by Horner's rule, the inclusive cutoff test, one exp2 and the two accumulations
// (numerator S, denominator W).  The four slots' partial sums of a voxel are added in a fixed order
// at the end, so the result is bitwise deterministic.
//
// Backward: one workgroup per group of G consecutive bricks (eight bricks and eight waves, or two or
// one brick and one wave), one Gaussian (key) per lane.  The bricks' per-voxel factors
// c_p = dL/dI(p) / (W(p) + eps) and I(p) are staged in LDS; the keys of the group's bricks are ordered
// together by their number of rows in their brick so that the lanes of a wave run similar numbers of
// iterations (more bricks give the ordering more keys to balance: 64-key batches cut from the keys of
// eight bricks are far more uniform than from two); each lane walks the rows of its Gaussian's box
// inside its brick in one flat loop, skips
// rows whose maximum exponent is below the cutoff, evaluates the BX voxels of a row unrolled, and
// accumulates per row the moments sum(k), sum(k ck), sum(k ck^2) and sum(c w) of k = dL/dw * w
// (ck: the voxel's x offset from the row's centre, so that dx = dxc + ck h with one dxc per key),
// folded with the row's (dy, dz) into the 11 brick-local sums of (1, delta, delta delta^T) and dA;
// the key's x moments follow from the ck moments at its end.
// The sums of each (Gaussian, brick) pair are written to the key's pre-sort slot; a second kernel
// reduces each Gaussian's slots in slot order and applies the chain rule (no atomics; deterministic).
#include <hip/hip_runtime.h>

#include <cmath>

#include "geom.h"
#include "gs_internal.h"

namespace gs {

// v of the lane N places along inside the lane's 16-lane DPP row (rotation).
template <int N>
__device__ __forceinline__ float dpp_row_ror(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x120 + N, 0xF, 0xF, false));
}

// Conservative test of one Gaussian against the 4x2x2-voxel cells of a BX x 8 x 4 brick.  Bit
// 4 q + c of the result is cell c = cy + 2 cz (cy, cz in {0, 1}) of quarter q = sx + (BX/4) sy, the
// cell spanning x in [x0 + 4 sx, +3], y in [y0 + 4 sy + 2 cy, +1], z in [z0 + 2 cz, +1].  Per z-pair
// slab the ellipsoid's x- and y-extents are taken (exact for the slab); a cell passes if a voxel
// centre of its x-range lies in the x-extent and a voxel centre of its y-range in the y-extent of its
// z-slab.  A voxel centre within the ellipsoid lies in the extents of the slab that contains it, so
// a cell holding a pair with d^2 <= 9 always passes.  (Adding the x-y coupling, i.e. the y-extent
// inside each x-slab, culls a few more cells but costs more than it saves.)
template <int BX>
__device__ __forceinline__ uint32_t cell_mask(const BrickGrid &bg, const EvalRec &e, const CullRec &c, float cutoff,
                                              int x0, int y0, int z0) {
  constexpr int NQX = BX / 4;
  if (c.c1.z == 0.f) return 0u;
  const float mx = e.r0.x, my = e.r0.y, mz = e.r0.z;
  const float sxx = c.c0.x, syy = c.c0.y, szz = c.c0.z, sxz = c.c1.x, syz = c.c1.y;
  const SlabAxes kxz = slab_axes(sxx, szz, sxz, cutoff), kyz = slab_axes(syy, szz, syz, cutoff);
  const float tx = extent_tol(mx, cutoff * __builtin_amdgcn_sqrtf(sxx), bg.hx),
              ty = extent_tol(my, cutoff * __builtin_amdgcn_sqrtf(syy), bg.hy);
  // x index range and y extent inside each z-pair slab
  int ixl[2], ixh[2];
  float yzl[2], yzh[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const float Z0 = centre(bg.oz, bg.hz, z0 + 2 * h), Z1 = centre(bg.oz, bg.hz, z0 + 2 * h + 1);
    float xl, xh;
    const bool okx = slab_extent(kxz, mx, mz, cutoff, Z0, Z1, tx, xl, xh);
    const bool oky = slab_extent(kyz, my, mz, cutoff, Z0, Z1, ty, yzl[h], yzh[h]);
    const bool ok = okx && oky;
    world_to_index(xl, xh, bg.ox, bg.ihx, bg.nx, ixl[h], ixh[h]);
    if (!ok) {
      ixl[h] = 1;
      ixh[h] = 0;
    }
  }
  uint32_t m = 0;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    int iyl, iyh;
    world_to_index(yzl[h], yzh[h], bg.oy, bg.ihy, bg.ny, iyl, iyh);
    const int pl = max(iyl - y0, 0) >> 1, ph = min(iyh - y0, 7) >> 1;
    const uint32_t pm0 = (iyl <= iyh && pl <= ph) ? (2u << ph) - (1u << pl) : 0u;
#pragma unroll
    for (int sx = 0; sx < NQX; ++sx) {
      const int xa = x0 + 4 * sx;
      const bool xin = ixl[h] <= ixh[h] && ixl[h] <= xa + 3 && ixh[h] >= xa;
      const uint32_t pm = xin ? pm0 : 0u;
      m |= ((pm & 3u) << (4 * sx + 2 * h)) | ((pm >> 2) << (4 * (sx + NQX) + 2 * h));
    }
  }
  return m;
}

// Origin (voxel indices) of the scan-local brick lb; brick counts are below 2^31 (checked when the
// scan table is built), so the 32-bit multiply-high division of the brick grid applies.
__device__ __forceinline__ void brick_coords(const BrickGrid &bg, int64_t lb, int &x0, int &y0, int &z0) {
  const uint32_t l = (uint32_t)lb, nbx = (uint32_t)bg.nbx, nby = (uint32_t)bg.nby;
  const uint32_t row = (__umulhi(l, bg.mbx) + l) >> bg.sbx, kz = (__umulhi(row, bg.mby) + row) >> bg.sby;
  const int kx = (int)(l - row * nbx), ky = (int)(row - kz * nby);
  x0 = kx << bg.lbx;
  y0 = ky * 8;
  z0 = kz * 4;
}

template <int BX, bool COUNT>
__global__ __launch_bounds__(32 * BX) void k_fwd(const ScanTable T, float cutoff, float eps,
                                                 const EvalRec *__restrict__ er, const CullRec *__restrict__ cr,
                                                 const uint32_t *__restrict__ list_gid,
                                                 const uint2 *__restrict__ brick_se, const DevStatus *st,
                                                 float *__restrict__ I, float *__restrict__ W,
                                                 unsigned long long *__restrict__ pair_count,
                                                 unsigned long long *__restrict__ eval_count) {
  constexpr int NT = 32 * BX, NW = BX / 2, NQX = BX / 4;
  if (st->overflow) return;
  // srec[NT] is an empty record (threshold +inf: never a pair) that pads the cell lists; the lists
  // hold byte offsets into srec
  __shared__ EvalRec srec[NT + 1];
  __shared__ uint32_t smask[NT];
  __shared__ uint16_t wlist[NW][4][NT + 4];
  constexpr uint16_t kPad = (uint16_t)(NT * sizeof(EvalRec));
  __shared__ unsigned long long scount[NW][3];

  const int64_t b = blockIdx.x;
  const ScanDesc &sd = T.s[T.of_brick(b)];
  const BrickGrid &bg = sd.bg;
  int x0, y0, z0;
  brick_coords(bg, b - sd.b0, x0, y0, z0);
  // wave w owns quarter w; its lane l = 16 g + 4 j + r works on cell g of the quarter (cy = g & 1,
  // cz = g >> 1), Gaussian slot j of the four in flight, and row r of the cell (ry = r & 1, rz = r >> 1)
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const int grp = l >> 4, sub = (l >> 2) & 3, r = l & 3;
  const int qx0 = x0 + (w % NQX) * 4;
  const int iy = y0 + (w / NQX) * 4 + 2 * (grp & 1) + (r & 1);
  const int iz = z0 + 2 * (grp >> 1) + (r >> 1);
  const float py = centre(bg.oy, bg.hy, iy), pz = centre(bg.oz, bg.hz, iz);
  float px[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) px[k] = centre(bg.ox, bg.hx, qx0 + k);
  const bool rowin = iy < bg.ny && iz < bg.nz;
  const uint2 se = brick_se[b];
  const uint32_t start = se.x, end = se.y;

  if (t == 0) {
    srec[NT].r0 = make_float4(0.f, 0.f, 0.f, 0.f);
    srec[NT].r1 = make_float4(0.f, 0.f, 0.f, INFINITY);
    srec[NT].r2 = make_float4(0.f, 0.f, 0.f, 0.f);
  }
  float Wa[4] = {0.f, 0.f, 0.f, 0.f}, Sa[4] = {0.f, 0.f, 0.f, 0.f};
  // COUNT: useful pairs, evaluated voxel slots of real list entries inside the grid, issued slots
  uint32_t npairs = 0, nevals = 0, nissued = 0;
  const uint32_t row_vox = rowin ? (uint32_t)max(0, min(4, bg.nx - qx0)) : 0u;
  for (uint32_t c0 = start; c0 < end; c0 += NT) {
    const int cnt = (int)min((uint32_t)NT, end - c0);
    if (t < cnt) {
      const uint32_t gid = list_gid[c0 + t];
      if (gid < T.n_total) {
        const EvalRec e = er[gid];
        const CullRec c = cr[gid];
        srec[t] = e;
        smask[t] = cell_mask<BX>(bg, e, c, cutoff, x0, y0, z0);
      } else {
        smask[t] = 0u;
      }
    }
    __syncthreads();
    // the wave's four cell lists, compacted in list order
    int n[4] = {0, 0, 0, 0};
    for (int j0 = 0; j0 < cnt; j0 += 64) {
      const int j = j0 + l;
      const uint32_t qm = j < cnt ? (smask[j] >> (4 * w)) & 15u : 0u;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const bool has = (qm >> g) & 1u;
        const uint64_t bal = __ballot(has);
        // the lane's rank among the wave's lanes that have the cell (lanes below it with the bit set)
        const uint32_t rank =
            __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
        if (has) wlist[w][g][n[g] + rank] = (uint16_t)(j * sizeof(EvalRec));
        n[g] += __popcll(bal);
      }
    }
    // every list padded with the empty record to the longest one, rounded up to a multiple of 4
    const int n4 = (max(max(n[0], n[1]), max(n[2], n[3])) + 3) & ~3;
#pragma unroll
    for (int g = 0; g < 4; ++g)
      for (int k = n[g] + l; k < n4; k += 64) wlist[w][g][k] = kPad;
    __syncthreads();
    const uint16_t *mylist = wlist[w][grp];
    for (int j0 = 0; j0 < n4; j0 += 4) {
      if (COUNT) {
        nevals += mylist[j0 + sub] != kPad ? row_vox : 0u;
        nissued += 4u;
      }
      const EvalRec R = *reinterpret_cast<const EvalRec *>(reinterpret_cast<const char *>(srec) + mylist[j0 + sub]);
      const float thr = R.r1.w;
      float dy, dz, bq, cq;
      row_coeffs(R, py, pz, dy, dz, bq, cq);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float q = row_q(R.r1.x, bq, cq, px[k] - R.r0.x);
        const bool in = q >= thr;
        if (COUNT) {
          npairs += (in && rowin && qx0 + k < bg.nx) ? 1u : 0u;
        } else {
          float wt = fast_exp2(q);
          wt = in ? wt : 0.f;
          Wa[k] += wt;
          Sa[k] = fmaf(R.r0.w, wt, Sa[k]);
        }
      }
    }
    // the next chunk reuses the staging areas; after the last one each wave goes on to its own
    // epilogue (which needs no LDS) without waiting for the others
    if (c0 + NT < end) __syncthreads();
  }
  if (COUNT) {
    unsigned long long v[3] = {npairs, nevals, nissued};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int d = 32; d > 0; d >>= 1) v[c] += __shfl_down(v[c], d, 64);
      if (l == 0) scount[w][c] = v[c];
    }
    __syncthreads();
    if (t < 3) {
      unsigned long long tot = 0;
      for (int k = 0; k < NW; ++k) tot += scount[k][t];
      if (t == 0) atomicAdd(pair_count, tot);
      else if (eval_count) atomicAdd(eval_count + (t - 1), tot);
    }
    return;
  }
  // the four slots' partial sums of each voxel of a row: rotations by 4 and then 8 lanes inside the
  // group's 16-lane DPP row add the slots in a fixed order per lane; lane j of the row then produces
  // voxel j (every voxel always comes from the same lane and the same order)
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    Wa[k] += dpp_row_ror<4>(Wa[k]);
    Sa[k] += dpp_row_ror<4>(Sa[k]);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    Wa[k] += dpp_row_ror<8>(Wa[k]);
    Sa[k] += dpp_row_ror<8>(Sa[k]);
  }
  const float Wv = sub == 0 ? Wa[0] : (sub == 1 ? Wa[1] : (sub == 2 ? Wa[2] : Wa[3]));
  const float Sv = sub == 0 ? Sa[0] : (sub == 1 ? Sa[1] : (sub == 2 ? Sa[2] : Sa[3]));
  if (rowin && qx0 + sub < bg.nx) {
    const int64_t v = sd.v0 + ((int64_t)iz * bg.ny + iy) * bg.nx + qx0 + sub;
    // hardware reciprocal (1 ulp): I within 2 ulp of S / (W + eps)
    I[v] = Sv * __builtin_amdgcn_rcpf(Wv + eps);
    if (W) W[v] = Wv;
  }
}

__global__ void k_zero_u64(unsigned long long *p) {
  if (threadIdx.x == 0) *p = 0ull;
}

template <bool COUNT>
static hipError_t fwd_dispatch(const ScanTable &T, int bx, float cutoff, float eps, const void *ws, const WsLayout &L,
                               float *I, float *W, unsigned long long *cnt, hipStream_t s,
                               unsigned long long *evals = nullptr) {
  const char *b = (const char *)ws;
  const unsigned nb = (unsigned)T.nbricks_total;
  if (nb == 0) return hipSuccess;
  const EvalRec *er = (const EvalRec *)(b + L.evalrec);
  const CullRec *cr = (const CullRec *)(b + L.cullrec);
  const uint32_t *lg = (const uint32_t *)(b + L.list_gid);
  const uint2 *bo = (const uint2 *)(b + L.brick_se);
  const DevStatus *st = (const DevStatus *)(b + L.status);
  switch (bx) {
    case 4: k_fwd<4, COUNT><<<nb, 128, 0, s>>>(T, cutoff, eps, er, cr, lg, bo, st, I, W, cnt, evals); break;
    case 8: k_fwd<8, COUNT><<<nb, 256, 0, s>>>(T, cutoff, eps, er, cr, lg, bo, st, I, W, cnt, evals); break;
    default: k_fwd<16, COUNT><<<nb, 512, 0, s>>>(T, cutoff, eps, er, cr, lg, bo, st, I, W, cnt, evals); break;
  }
  return hipGetLastError();
}

hipError_t launch_fwd(const ScanTable &T, int bx, float cutoff, float eps, const void *ws, const WsLayout &L,
                      float *I, float *W, hipStream_t s) {
  prof_begin(s);
  hipError_t e = fwd_dispatch<false>(T, bx, cutoff, eps, ws, L, I, W, nullptr, s);
  prof_end(s, "render_fwd");
  return e;
}

hipError_t launch_count_pairs(const ScanTable &T, int bx, float cutoff, const void *ws, const WsLayout &L,
                              int64_t *d_count, hipStream_t s) {
  prof_begin(s);
  k_zero_u64<<<1, 64, 0, s>>>((unsigned long long *)d_count);
  hipError_t e = fwd_dispatch<true>(T, bx, cutoff, 0.f, ws, L, nullptr, nullptr, (unsigned long long *)d_count, s);
  prof_end(s, "count_pairs");
  return e;
}

// ------------------------------------------------------------------------------------------------
// Backward, brick-local partial sums.  Partial record of one (Gaussian, brick) key, 3 x float4:
//   p0 = (sum c w, sum k, sum k dx, sum k dy), p1 = (sum k dz, sum k dx dx, sum k dy dy, sum k dz dz),
//   p2 = (sum k dx dy, sum k dx dz, sum k dy dz, 0)
// with c = dL/dI / (W + eps), k = c (A - I) w = dL/dw * w.

constexpr int kBwdWave = 64;  // lanes per wave; a backward workgroup has NW waves
// ordering buckets: full-row keys by rows in the brick (32 .. 0, bucket 0 = 32 rows), half-row keys
// likewise (buckets 33 ..), then empty boxes
constexpr int kBwdBuckets = 67;

// FIT: the fit's loss is fused into the staging.  The brick's 4 z slices are one group of the
// z-mean (LR slice z0 / 4): per (x, y) column, LR = (((I0 + I1) + I2) + I3) * 1/4 (the loss kernel's
// order), dL/dI = sign(LR - obs) * gscale on the column's 4 voxels, and the brick's sum of |LR - obs|
// goes to loss_part[brick] (also for bricks without Gaussians).  Otherwise dL/dI is read from gI.
template <int BX, bool FIT>
__device__ __forceinline__ void bwd_stage(const ScanDesc &sd, int64_t b, int x0, int y0, int z0, int t,
                                          const float *__restrict__ Iv, const float *__restrict__ Wv,
                                          const float *__restrict__ gI, const float *__restrict__ obs, float eps,
                                          float *__restrict__ loss_part, float2 *sCI) {
  constexpr int RP = BX + 1;
  const BrickGrid &bg = sd.bg;
  if (FIT) {
    // BX * 8 columns of 4 voxels, one per thread and pass
    float absd = 0.f;
    for (int col = t; col < BX * 8; col += kBwdWave) {
      const int lx = col % BX, ly = col / BX;
      const int gx = x0 + lx, gy = y0 + ly;
      float c4[4] = {0.f, 0.f, 0.f, 0.f}, i4[4] = {0.f, 0.f, 0.f, 0.f};
      if (gx < bg.nx && gy < bg.ny) {
        const int64_t plane = (int64_t)bg.nx * bg.ny;
        const int64_t g0 = sd.v0 + ((int64_t)z0 * bg.ny + gy) * bg.nx + gx;
#pragma unroll
        for (int z = 0; z < 4; ++z) i4[z] = Iv[g0 + z * plane];
        const float lr = (((i4[0] + i4[1]) + i4[2]) + i4[3]) * 0.25f;
        const float d = lr - obs[sd.o0 + ((int64_t)(z0 >> 2) * bg.ny + gy) * bg.nx + gx];
        const float sg = d > 0.f ? sd.gscale : (d < 0.f ? -sd.gscale : 0.f);
        absd += fabsf(d);
#pragma unroll
        for (int z = 0; z < 4; ++z) c4[z] = sg / (Wv[g0 + z * plane] + eps);
      }
#pragma unroll
      for (int z = 0; z < 4; ++z) sCI[(z * 8 + ly) * RP + lx] = make_float2(c4[z], i4[z]);
    }
    // the brick's loss sum: each thread's columns in order, then a fixed-order wave reduction
    float wsum = absd;
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) wsum += __shfl_down(wsum, d, 64);
    if (t == 0) loss_part[b] = wsum;
  } else {
    // per voxel of the brick: c = dL/dI / (W + eps) and I; zero outside the grid, so that voxels
    // beyond the grid's edge contribute nothing
    for (int v = t; v < BX * 32; v += kBwdWave) {
      const int lx = v % BX, ly = (v / BX) & 7, lz = v / (BX * 8);
      const int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
      float c = 0.f, iv = 0.f;
      if (gx < bg.nx && gy < bg.ny && gz < bg.nz) {
        const int64_t g = sd.v0 + ((int64_t)gz * bg.ny + gy) * bg.nx + gx;
        c = gI[g] / (Wv[g] + eps);
        iv = Iv[g];
      }
      sCI[(lz * 8 + ly) * RP + lx] = make_float2(c, iv);
    }
  }
}

// The 11 brick-local sums of one key (see the partial record above), with the x moments kept as
// moments of ck, the voxel's x offset from the centre of the evaluated row segment.
struct KeySums {
  float sA, sk, sc, sky, skz, scc, myy, mzz, scy, scz, myz;
};

// The rows of one key's box in its brick (nrows rows, y fastest over [yl, yh] x [zl, zh]), each
// evaluated over W voxels starting at the global voxel index xw: the whole brick row (W = BX), or a
// window of BX/2 voxels that holds the key's x-range in the brick (the voxels left out lie outside
// its box, so they hold no pair).  Per row, the quadratic's maximum along x (at dx* = -b / 2a) is
// compared with the cutoff with a rounding allowance, so a row holding a pair with d^2 <= 9 is never
// skipped; a live row's voxels are evaluated unrolled with the forward's per-pair predicate into
// sum c w, sum k, sum k ck, sum k ck^2, which are folded with the row's (dy, dz).  ck = kk - (W-1)/2
// is a compile-time constant, so dx = dxc + ck h with one dxc per key (returned): the x moments follow
// from the ck moments (sum k dx = dxc sum k + h sum k ck, ...), a multiply per voxel less than
// accumulating k dx and k dx^2.  COUNT: only counts the evaluated and issued voxel slots.
template <int W, bool COUNT>
__device__ __forceinline__ float key_rows(const BrickGrid &bg, const EvalRec &R, int xw, const float2 *sC, int RP,
                                          const float *sPy, const float *sPz, int yl, int yh, int zl, int nrows,
                                          KeySums &s, uint32_t &c_eval, uint32_t &c_issued) {
  const float mx = R.r0.x, A = R.r0.w;
  const float a = R.r1.x, thr = R.r1.w;  // Q_xx < 0
  float px[W];
#pragma unroll
  for (int kk = 0; kk < W; ++kk) px[kk] = centre(bg.ox, bg.hx, xw + kk);
  s = KeySums{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  const float inv4a = 0.25f * __builtin_amdgcn_rcpf(a);
  const float thr_lo = thr - 1e-5f * (1.f + fabsf(thr));  // the row test's allowance, key part
  int iy = yl, iz = zl;
  for (int r = 0; r < nrows; ++r) {
    const float py = sPy[iy], pz = sPz[iz];
    float dy, dz, bq, cq;
    row_coeffs(R, py, pz, dy, dz, bq, cq);
    // the row's maximum of q (at dx* = -b / (2a)) is c - b^2 / (4a); rows whose maximum is clearly
    // below the cutoff hold no pair
    const float qmax = fmaf(-(bq * bq), inv4a, cq);
    const bool live = qmax >= fmaf(-1e-5f, fabsf(cq), thr_lo);
    if (COUNT) {
      c_eval += live ? (uint32_t)W : 0u;
      c_issued += __ballot(live) != 0ull && lane_id() == __builtin_amdgcn_readfirstlane(lane_id())
                      ? (uint32_t)(64 * W)
                      : 0u;
    } else if (live) {
      const int rb = (iz * 8 + iy) * RP;
      float tA, m0, m1, m2;
#pragma unroll
      for (int kk = 0; kk < W; ++kk) {
        constexpr float half = 0.5f * (W - 1);
        const float ck = (float)kk - half;
        const float dx = px[kk] - mx;
        const float qv = row_q(a, bq, cq, dx);
        float wt = fast_exp2(qv);
        wt = qv >= thr ? wt : 0.f;
        const float2 ci = sC[rb + kk];
        const float tt = ci.x * wt;
        const float kap = (A - ci.y) * tt;
        if (kk == 0) {  // the row's sums start from the first voxel's terms
          tA = tt;
          m0 = kap;
          m1 = ck * kap;
          m2 = (ck * ck) * kap;
        } else {
          tA += tt;
          m0 += kap;
          m1 = fmaf(ck, kap, m1);
          m2 = fmaf(ck * ck, kap, m2);
        }
      }
      s.sA += tA;
      s.sk += m0;
      s.sc += m1;
      s.sky = fmaf(m0, dy, s.sky);
      s.skz = fmaf(m0, dz, s.skz);
      s.scc += m2;
      s.scy = fmaf(m1, dy, s.scy);
      s.scz = fmaf(m1, dz, s.scz);
      const float m0dy = m0 * dy;
      s.myy = fmaf(m0dy, dy, s.myy);
      s.myz = fmaf(m0dy, dz, s.myz);
      s.mzz = fmaf(m0 * dz, dz, s.mzz);
    }
    if (++iy > yh) {
      iy = yl;
      ++iz;
    }
  }
  return fmaf(0.5f * (W - 1), bg.hx, px[0] - mx);  // dxc: the segment centre's x offset
}

// Backward modes: plain (dL/dI given), fit (loss fused into the staging), count (the ordering and
// the row tests only, counting evaluated and issued voxel slots; nothing is written but the counts).
constexpr int kBwdPlain = 0, kBwdFit = 1, kBwdCount = 2;

// One workgroup of NW waves per group of G consecutive bricks of a scan.  Wave w stages the bricks
// j = w, w + NW, ... of the group (as a single wave: the fit's per-brick loss sums do not depend on the
// workgroup shape).  The keys of all G bricks are ordered together, WIN at a time, by class (full
// rows, then half rows) and number of rows; the waves take the ordered keys 64 at a time, wave w
// batch w first and then whichever batch is next when it is done (an LDS counter), so that the
// heaviest batches start first and the lighter ones fill in.  Eight-wave groups of bricks up to 8 wide have their registers
// capped for 8 waves per SIMD, i.e. four workgroups per CU, so that the memory-bound phases of some
// workgroups (staging, ordering, the partial sums' stores) overlap the VALU-bound row loops of others.
template <int BX, int MODE, int G, int WIN, int NW>
__global__ __launch_bounds__(kBwdWave *NW) __attribute__((amdgpu_waves_per_eu(NW == 8 && BX <= 8 ? 8 : 1)))
void k_bwd(const ScanTable T, float eps, const EvalRec *__restrict__ er, const uint4 *__restrict__ gbox,
           const uint32_t *__restrict__ list_gid, const uint32_t *__restrict__ list_slot,
           const uint2 *__restrict__ brick_se, const DevStatus *st, const float *__restrict__ Iv,
           const float *__restrict__ Wv, const float *__restrict__ gI, const float *__restrict__ obs,
           float *__restrict__ loss_part, int64_t cap, float4 *__restrict__ part,
           unsigned long long *__restrict__ eval_count) {
  constexpr bool FIT = MODE == kBwdFit, COUNT = MODE == kBwdCount;
  constexpr int NT = kBwdWave * NW;
  constexpr int RP = BX + 1;  // LDS row stride in voxels (pad: rows of a wave hit different banks)
  // LDS voxels per brick, padded so that the same row of different bricks falls into different banks
  // (keys of similar boxes in the bricks read the same row index at the same time)
  constexpr int BV = 32 * RP + 4;
  static_assert(G <= 8, "the brick of a key takes 3 bits of its box word");
  if (st->overflow) return;
  __shared__ float2 sCI[G * BV];
  __shared__ uint16_t sorder[WIN];
  __shared__ uint8_t sbucket[WIN];
  // key's box in its brick: yl, yh (3 bits each), zl, zh (2 bits each), brick of the group (bits
  // 10-12), xl, xh (4 bits each, bits 13-20), empty (bit 21)
  __shared__ uint32_t sbox[WIN];
  __shared__ uint32_t bcount[kBwdBuckets], bcursor[kBwdBuckets];
  __shared__ int sorg[G][3];  // brick origins (voxel indices)
  __shared__ float spy[G][8], spz[G][4];  // voxel-centre coordinates of the bricks' rows and slices
  // boff[j]: where brick j's keys start in the group's contiguous key range (for a brick without
  // keys, where the next brick's start), boff[G]: the range's end
  __shared__ uint32_t sboff[G + 1];
  __shared__ uint32_t snext;  // the window's next 64-key batch to hand out (batch w starts wave w)
  __shared__ uint2 sse[G];
  const int64_t q = blockIdx.x;
  const ScanDesc &sd = T.s[T.of_group(q)];
  const BrickGrid &bg = sd.bg;
  const int64_t lb = G * (q - sd.p0);  // the group's first brick, scan-local
  const int nbk = (int)min((int64_t)G, bg.nbricks - lb);
  const int64_t b = sd.b0 + lb;
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  if (t < G) {
    int x0, y0, z0;
    brick_coords(bg, lb + min(t, nbk - 1), x0, y0, z0);
    sorg[t][0] = x0;
    sorg[t][1] = y0;
    sorg[t][2] = z0;
    sse[t] = t < nbk ? brick_se[b + t] : make_uint2(0u, 0u);
  }
  if (t < 8 * G) {
    const int j = t / 8;
    int x0, y0, z0;
    brick_coords(bg, lb + min(j, nbk - 1), x0, y0, z0);
    spy[j][t % 8] = centre(bg.oy, bg.hy, y0 + t % 8);
    if (t % 8 < 4) spz[j][t % 8] = centre(bg.oz, bg.hz, z0 + t % 8);
  }
  __syncthreads();
  if (t == 0) {
    uint32_t e = 0u;
    for (int j = 0; j < G; ++j) e = max(e, sse[j].y);
    sboff[G] = e;
    for (int j = G - 1; j >= 0; --j) sboff[j] = sse[j].y > sse[j].x ? sse[j].x : sboff[j + 1];
  }
  // COUNT: voxel slots of rows passing the row test, issued lane-voxel slots, rows in the boxes
  uint32_t c_eval = 0, c_issued = 0, c_rows = 0;
  if (!COUNT) {
    for (int j = w; j < nbk; j += NW) {
      if (FIT || sse[j].y > sse[j].x)
        bwd_stage<BX, FIT>(sd, b + j, sorg[j][0], sorg[j][1], sorg[j][2], l, Iv, Wv, gI, obs, eps, loss_part,
                           sCI + j * BV);
    }
  }
  __syncthreads();
  const uint32_t start = sboff[0], end = sboff[G];
  if (start == end) return;
  (void)c_eval;
  (void)c_issued;
  (void)c_rows;
  for (uint32_t w0 = start; w0 < end; w0 += WIN) {
    const int L = (int)min((uint32_t)WIN, end - w0);
    // order the window's keys (of all bricks of the group) by their number of rows in their brick,
    // most first, so that the lanes of a wave run similar numbers of row iterations (each key's
    // result is independent of where it runs, so the order does not change any result)
    for (int k = t; k < kBwdBuckets; k += NT) bcount[k] = 0u;
    if (t == 0) snext = NW;
    __syncthreads();
    for (int j = t; j < L; j += NT) {
      const uint32_t k = w0 + j;
      const uint32_t gid = list_gid[k];
      int kb = 0;
#pragma unroll
      for (int g = 1; g < G; ++g) kb += k >= sboff[g] ? 1 : 0;
      const int xb = sorg[kb][0], yb = sorg[kb][1], zb = sorg[kb][2];
      const int xeb = min(xb + BX - 1, bg.nx - 1), yeb = min(yb + 7, bg.ny - 1), zeb = min(zb + 3, bg.nz - 1);
      int bk = kBwdBuckets - 1;
      uint32_t box = (1u << 21) | ((uint32_t)kb << 10);  // empty
      if (gid < T.n_total) {
        // the Gaussian's voxel box (its padded 3-sigma extent, from the prep) clipped to the brick
        const uint4 vb = gbox[gid];
        const int xl = max((int)(vb.x & 0xFFFFu), xb), xh = min((int)(vb.x >> 16), xeb);
        const int yl = max((int)(vb.y & 0xFFFFu), yb), yh = min((int)(vb.y >> 16), yeb);
        const int zl = max((int)(vb.z & 0xFFFFu), zb), zh = min((int)(vb.z >> 16), zeb);
        if (xl <= xh && yl <= yh && zl <= zh) {
          // full-row keys first, then the half-row keys (each class by rows, most first)
          const bool narrow = BX > 4 && xh - xl < BX / 2;
          bk = (narrow ? 33 : 0) + 32 - (yh - yl + 1) * (zh - zl + 1);
          box = (uint32_t)((yl - yb) | ((yh - yb) << 3) | ((zl - zb) << 6) | ((zh - zb) << 8) | (kb << 10) |
                           ((xl - xb) << 13) | ((xh - xb) << 17));
        }
      }
      sbucket[j] = (uint8_t)bk;
      sbox[j] = box;
      atomicAdd(&bcount[bk], 1u);
    }
    __syncthreads();
    if (t == 0) {
      uint32_t run = 0;
      for (int k = 0; k < kBwdBuckets; ++k) {
        bcursor[k] = run;
        run += bcount[k];
      }
    }
    __syncthreads();
    for (int j = t; j < L; j += NT) sorder[atomicAdd(&bcursor[sbucket[j]], 1u)] = (uint16_t)j;
    __syncthreads();
    for (int r = 0;; ++r) {
      // batch w first, then whichever batch is next in line when the wave is done with its last:
      // the batches come heaviest first, so this is longest-first list scheduling over the waves
      uint32_t bi = (uint32_t)w;
      if (r > 0) {
        const uint32_t v = l == 0 ? atomicAdd(&snext, 1u) : 0u;
        bi = (uint32_t)__shfl((int)v, 0, 64);
      }
      const int c0 = kBwdWave * (int)bi;
      if (c0 >= L) break;  // uniform per wave
      const int p = c0 + l;
      if (p >= L) continue;
      const int jj = sorder[p];
      const uint32_t k = w0 + jj;
      const uint32_t gid = list_gid[k];
      const uint32_t slot = list_slot[k];
      if (gid >= T.n_total || (int64_t)slot >= cap) continue;
      const EvalRec R = er[gid];
      const uint32_t box = sbox[jj];
      const int kb = (box >> 10) & 7;
      const int bx0 = sorg[kb][0];
      const float2 *sC = sCI + kb * BV;
      const float *sPy = spy[kb], *sPz = spz[kb];
      // the box in brick-local rows and slices
      const int yl = box & 7, yh = (box >> 3) & 7, zl = (box >> 6) & 3, zh = (box >> 8) & 3;
      // keys whose x-range in the brick fits half a brick row evaluate that half only (one of two
      // code paths per key, whatever the batch: a key's sums do not depend on where it runs)
      const int xl = (box >> 13) & 15, xh = (box >> 17) & 15;
      const bool narrow = BX > 4 && xh - xl < BX / 2;
      const int nrows = (box >> 21) ? 0 : (yh - yl + 1) * (zh - zl + 1);
      if (COUNT) c_rows += (uint32_t)nrows;
      KeySums s;
      float dxc;
      if (narrow)
        dxc = key_rows<BX / 2, COUNT>(bg, R, bx0 + min(xl, BX / 2), sC + min(xl, BX / 2), RP, sPy, sPz, yl, yh, zl,
                                      nrows, s, c_eval, c_issued);
      else
        dxc = key_rows<BX, COUNT>(bg, R, bx0, sC, RP, sPy, sPz, yl, yh, zl, nrows, s, c_eval, c_issued);
      if (COUNT) continue;
      // back from segment-centre offsets to dx: sum k dx = dxc sum k + h sum ck k, sum k dx^2 =
      // dxc^2 sum k + 2 dxc h sum ck k + h^2 sum ck^2 k, sum k dx d = dxc sum k d + h sum ck k d
      const float hx = bg.hx;
      const float skx = fmaf(hx, s.sc, dxc * s.sk);
      const float mxx = fmaf(dxc, fmaf(dxc, s.sk, 2.f * hx * s.sc), (hx * hx) * s.scc);
      const float mxy = fmaf(hx, s.scy, dxc * s.sky);
      const float mxz = fmaf(hx, s.scz, dxc * s.skz);
      float4 *o = part + (int64_t)slot * 3;
      o[0] = make_float4(s.sA, s.sk, skx, s.sky);
      o[1] = make_float4(s.skz, mxx, s.myy, s.mzz);
      o[2] = make_float4(mxy, mxz, s.myz, 0.f);
    }
    __syncthreads();
  }
  if (COUNT) {
    unsigned long long v[3] = {c_eval, c_issued, c_rows};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int d = 32; d > 0; d >>= 1) v[c] += __shfl_down(v[c], d, 64);
    }
    if (l == 0) {
      atomicAdd(eval_count + 0, v[0]);
      atomicAdd(eval_count + 1, v[1]);
      atomicAdd(eval_count + 2, v[2]);
    }
  }
}

template <int MODE, int G, int WIN, int NW>
static void bwd_launch(const ScanTable &T, int bx, float eps, const EvalRec *er, const uint4 *gb,
                       const uint32_t *lg, const uint32_t *ls, const uint2 *bo, const DevStatus *st, const float *I,
                       const float *W, const float *gI, const float *obs, float *loss_part, int64_t cap, float4 *part,
                       unsigned long long *evals, hipStream_t s) {
  const unsigned nb = (unsigned)T.ngroups_total;  // one workgroup per group of bricks
  switch (bx) {
    case 4:
      k_bwd<4, MODE, G, WIN, NW><<<nb, kBwdWave * NW, 0, s>>>(T, eps, er, gb, lg, ls, bo, st, I, W, gI, obs,
                                                               loss_part, cap, part, evals);
      break;
    case 8:
      k_bwd<8, MODE, G, WIN, NW><<<nb, kBwdWave * NW, 0, s>>>(T, eps, er, gb, lg, ls, bo, st, I, W, gI, obs,
                                                               loss_part, cap, part, evals);
      break;
    default:
      k_bwd<16, MODE, G, WIN, NW><<<nb, kBwdWave * NW, 0, s>>>(T, eps, er, gb, lg, ls, bo, st, I, W, gI, obs,
                                                                loss_part, cap, part, evals);
      break;
  }
}

// Group shapes: (G bricks, NW waves) = (8, 8) by default (a wave stages one brick), (2, 1) or (1, 1)
// by flag.  The ordering window holds 2048 keys for the eight-brick group and 512 for the others, or
// half as many with GS_FLAG_BWD_WINDOW_256.
template <int MODE>
static hipError_t bwd_dispatch(const ScanTable &T, int bx, uint32_t flags, float eps, const void *ws,
                               const WsLayout &L, const float *I, const float *W, const float *gI, const float *obs,
                               float *loss_part, hipStream_t s, unsigned long long *evals = nullptr) {
  char *b = (char *)ws;
  if (T.ngroups_total == 0) return hipSuccess;
  const EvalRec *er = (const EvalRec *)(b + L.evalrec);
  const uint4 *gb = (const uint4 *)(b + L.gbox);
  const uint32_t *lg = (const uint32_t *)(b + L.list_gid), *ls = (const uint32_t *)(b + L.list_slot);
  const uint2 *bo = (const uint2 *)(b + L.brick_se);
  const DevStatus *st = (const DevStatus *)(b + L.status);
  float4 *part = MODE == kBwdCount ? nullptr : (float4 *)(b + L.partials);
  const bool w256 = (flags & GS_FLAG_BWD_WINDOW_256) != 0;
#define GS_BWD_ARGS T, bx, eps, er, gb, lg, ls, bo, st, I, W, gI, obs, loss_part, L.cap, part, evals, s
  switch (T.bwd_bricks) {
    case 1:
      if (w256) bwd_launch<MODE, 1, 256, 1>(GS_BWD_ARGS);
      else bwd_launch<MODE, 1, 512, 1>(GS_BWD_ARGS);
      break;
    case 2:
      if (w256) bwd_launch<MODE, 2, 256, 1>(GS_BWD_ARGS);
      else bwd_launch<MODE, 2, 512, 1>(GS_BWD_ARGS);
      break;
    default:
      if (w256) bwd_launch<MODE, 8, 1024, 8>(GS_BWD_ARGS);
      else bwd_launch<MODE, 8, 2048, 8>(GS_BWD_ARGS);
      break;
  }
#undef GS_BWD_ARGS
  return hipGetLastError();
}

hipError_t launch_bwd(const ScanTable &T, int bx, uint32_t flags, float cutoff, float eps, void *ws, const WsLayout &L,
                      const float *I, const float *W, const float *dLdI, hipStream_t s) {
  prof_begin(s);
  hipError_t e = bwd_dispatch<kBwdPlain>(T, bx, flags, eps, ws, L, I, W, dLdI, nullptr, nullptr, s);
  prof_end(s, "render_bwd");
  return e;
}

hipError_t launch_bwd_fit(const ScanTable &T, int bx, uint32_t flags, float cutoff, float eps, void *ws,
                          const WsLayout &L, const float *I, const float *W, const float *obs, float *loss_part,
                          hipStream_t s) {
  prof_begin(s);
  hipError_t e = bwd_dispatch<kBwdFit>(T, bx, flags, eps, ws, L, I, W, nullptr, obs, loss_part, s);
  prof_end(s, "render_bwd");
  return e;
}

__global__ void k_zero_u64_n(unsigned long long *p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

hipError_t launch_count_evals(const ScanTable &T, int bx, uint32_t flags, float cutoff, const void *ws,
                              const WsLayout &L, int64_t *d_counts, hipStream_t s) {
  prof_begin(s);
  unsigned long long *c = (unsigned long long *)d_counts;
  k_zero_u64_n<<<1, 64, 0, s>>>(c, kEvalCounts);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = fwd_dispatch<true>(T, bx, cutoff, 0.f, ws, L, nullptr, nullptr, c, s, c + 1);
  if (e == hipSuccess)
    e = bwd_dispatch<kBwdCount>(T, bx, flags, 0.f, ws, L, nullptr, nullptr, nullptr, nullptr, nullptr, s,
                                c + 3);
  prof_end(s, "count_evals");
  return e;
}

}  // namespace gs
