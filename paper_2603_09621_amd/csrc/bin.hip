// Binning: per-Gaussian records, (brick, Gaussian) key generation with a conservative ellipsoid
// cull, and an LSD radix sort of the keys on brick id.
//
// The paper's rasterizer partitions the volume into bricks and, for each brick, identifies the
// Gaussians whose 3-sigma Mahalanobis ellipsoid meets it (§3.3).  Here every Gaussian enumerates the
// bricks its ellipsoid may meet: a count pass (fused with the record computation), an exclusive scan
// that numbers the keys Gaussian-major, and an emit pass that writes (brick id, Gaussian) at each key's
// slot.  A stable LSD radix sort on brick id (8-bit digits) then yields per-brick lists in ascending
// Gaussian order together with each key's slot, which the backward uses to store its partial sums;
// its last pass also records where each brick's list starts and ends.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "geom.h"
#include "gs_internal.h"

namespace gs {

// ------------------------------------------------------------------------------------------------
// Prep: (mu, s, q, A, r) -> evaluation and culling records (§3.1 parameters; §3.2 weight).  The
// records are built by a device function shared by the fused prep + count kernel.

// Returns false (and an empty record that yields no keys and no pairs) for a non-finite parameter,
// a zero quaternion or r <= 0.
__device__ __forceinline__ bool make_records(int64_t i, const float *__restrict__ mu, const float *__restrict__ ls,
                                             const float *__restrict__ quat, const float *__restrict__ amp,
                                             const float *__restrict__ relax, float cutoff, EvalRec &e, CullRec &cr) {
  float mx = mu[3 * i], my = mu[3 * i + 1], mz = mu[3 * i + 2];
  float s0 = ls[3 * i], s1 = ls[3 * i + 1], s2 = ls[3 * i + 2];
  float qw = quat[4 * i], qx = quat[4 * i + 1], qy = quat[4 * i + 2], qz = quat[4 * i + 3];
  float A = amp[i];
  float r = relax ? relax[i] : 1.f;
  float qn2 = qw * qw + qx * qx + qy * qy + qz * qz;
  bool ok = isfinite(mx) && isfinite(my) && isfinite(mz) && isfinite(s0) && isfinite(s1) && isfinite(s2) &&
            isfinite(qn2) && qn2 > 0.f && isfinite(A) && isfinite(r) && r > 0.f;
  if (!ok) {
    e = EvalRec{make_float4(0, 0, 0, 0), make_float4(0, 0, 0, 0), make_float4(0, 0, 0, 0)};
    cr = CullRec{make_float4(1, 1, 1, 0), make_float4(0, 0, 0, 0)};
    return false;
  }
  float qn = sqrtf(qn2);
  float w = qw / qn, x = qx / qn, y = qy / qn, z = qz / qn;
  float R[3][3] = {{1.f - 2.f * (y * y + z * z), 2.f * (x * y - w * z), 2.f * (x * z + w * y)},
                   {2.f * (x * y + w * z), 1.f - 2.f * (x * x + z * z), 2.f * (y * z - w * x)},
                   {2.f * (x * z - w * y), 2.f * (y * z + w * x), 1.f - 2.f * (x * x + y * y)}};
  float ev[3] = {expf(2.f * s0), expf(2.f * s1), expf(2.f * s2)};
  float iv[3] = {expf(-2.f * s0), expf(-2.f * s1), expf(-2.f * s2)};
  float S[3][3], P[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      S[a][b] = R[a][0] * ev[0] * R[b][0] + R[a][1] * ev[1] * R[b][1] + R[a][2] * ev[2] * R[b][2];
      P[a][b] = R[a][0] * iv[0] * R[b][0] + R[a][1] * iv[1] * R[b][1] + R[a][2] * iv[2] * R[b][2];
    }
  const float k = -kHalfLog2e;
  const float l2r = log2f(r);
  e.r0 = make_float4(mx, my, mz, A);
  e.r1 = make_float4(k * P[0][0], 2.f * k * P[0][1], 2.f * k * P[0][2], k * cutoff * cutoff + l2r);
  e.r2 = make_float4(k * P[1][1], 2.f * k * P[1][2], k * P[2][2], l2r);
  cr = CullRec{make_float4(S[0][0], S[1][1], S[2][2], S[0][1]), make_float4(S[0][2], S[1][2], 1.f, 0.f)};
  return true;
}

// ------------------------------------------------------------------------------------------------
// Key generation.  For one Gaussian: its axis-aligned 3-sigma voxel box; for each brick z-slab the
// y-extent of the ellipsoid inside that slab; for each brick row the x-extent inside the row's y-slab
// intersected with the x-extent inside the z-slab.  Every brick whose voxel centres fall in these
// conservative ranges receives a key.  The keys come in runs of consecutive bricks along x (one run
// per brick row), numbered z-slab by z-slab and row by row.  The same three functions below serve the
// per-lane enumeration of a Gaussian and the wave-wide one of a large Gaussian, so both give the
// same runs.

// A Gaussian's voxel box and the slab-independent parts of its three projections.
struct GaussBox {
  int xl, xh, yl, yh, zl, zh;
  SlabAxes kyz, kxz, kxy;
  float tx, ty;
};

__device__ __forceinline__ bool gauss_box(const BrickGrid &bg, const EvalRec &e, const CullRec &c, float cutoff,
                                          GaussBox &B) {
  if (c.c1.z == 0.f) return false;  // invalid Gaussian: no keys
  const float mx = e.r0.x, my = e.r0.y, mz = e.r0.z;
  const float sxx = c.c0.x, syy = c.c0.y, szz = c.c0.z, sxy = c.c0.w, sxz = c.c1.x, syz = c.c1.y;
  const float ex = cutoff * __builtin_amdgcn_sqrtf(sxx), ey = cutoff * __builtin_amdgcn_sqrtf(syy),
              ez = cutoff * __builtin_amdgcn_sqrtf(szz);
  B.tx = extent_tol(mx, ex, bg.hx);
  B.ty = extent_tol(my, ey, bg.hy);
  const float tz = extent_tol(mz, ez, bg.hz);
  world_to_index(mx - ex - B.tx, mx + ex + B.tx, bg.ox, bg.ihx, bg.nx, B.xl, B.xh);
  world_to_index(my - ey - B.ty, my + ey + B.ty, bg.oy, bg.ihy, bg.ny, B.yl, B.yh);
  world_to_index(mz - ez - tz, mz + ez + tz, bg.oz, bg.ihz, bg.nz, B.zl, B.zh);
  if (B.xl > B.xh || B.yl > B.yh || B.zl > B.zh) return false;
  B.kyz = slab_axes(syy, szz, syz, cutoff);
  B.kxz = slab_axes(sxx, szz, sxz, cutoff);
  B.kxy = slab_axes(sxx, syy, sxy, cutoff);
  return true;
}

// Brick z-slab kz of the box: the ellipsoid's voxel rows (y index range) and x extent inside it.
__device__ __forceinline__ bool slab_part(const BrickGrid &bg, const EvalRec &e, const GaussBox &B, float cutoff,
                                          int kz, int &yl2, int &yh2, float &xzlo, float &xzhi) {
  const int za = max(B.zl, kz << bg.lbz), zb = min(B.zh, ((kz + 1) << bg.lbz) - 1);
  const float Z0 = centre(bg.oz, bg.hz, za), Z1 = centre(bg.oz, bg.hz, zb);
  float ylo, yhi;
  if (!slab_extent(B.kyz, e.r0.y, e.r0.z, cutoff, Z0, Z1, B.ty, ylo, yhi)) return false;
  if (!slab_extent(B.kxz, e.r0.x, e.r0.z, cutoff, Z0, Z1, B.tx, xzlo, xzhi)) return false;
  world_to_index(ylo, yhi, bg.oy, bg.ihy, bg.ny, yl2, yh2);
  yl2 = max(yl2, B.yl);
  yh2 = min(yh2, B.yh);
  return yl2 <= yh2;
}

// Brick row ky of that slab (ky within [yl2 >> lby, yh2 >> lby]): its run of bricks [kx0, kx1].
__device__ __forceinline__ bool row_part(const BrickGrid &bg, const EvalRec &e, const GaussBox &B, float cutoff,
                                         int ky, int yl2, int yh2, float xzlo, float xzhi, int &kx0, int &kx1) {
  const int ya = max(yl2, ky << bg.lby), yb = min(yh2, ((ky + 1) << bg.lby) - 1);
  const float Y0 = centre(bg.oy, bg.hy, ya), Y1 = centre(bg.oy, bg.hy, yb);
  float xylo, xyhi;
  if (!slab_extent(B.kxy, e.r0.x, e.r0.y, cutoff, Y0, Y1, B.tx, xylo, xyhi)) return false;
  int xl2, xh2;
  world_to_index(fmaxf(xzlo, xylo), fminf(xzhi, xyhi), bg.ox, bg.ihx, bg.nx, xl2, xh2);
  xl2 = max(xl2, B.xl);
  xh2 = min(xh2, B.xh);
  if (xl2 > xh2) return false;
  kx0 = xl2 >> bg.lbx;
  kx1 = xh2 >> bg.lbx;
  return true;
}

// Brick rows (z-slab, y-row pairs) of the box: the work items of the wave-wide enumeration.
__device__ __forceinline__ uint32_t box_rows(const BrickGrid &bg, const GaussBox &B, uint32_t &nky) {
  nky = (uint32_t)((B.yh >> bg.lby) - (B.yl >> bg.lby) + 1);
  return nky * (uint32_t)((B.zh >> bg.lbz) - (B.zl >> bg.lbz) + 1);
}

// Run of box row r (row-major over (z-slab, y-row), the order of the per-lane enumeration); 0 keys
// if the ellipsoid misses the row.
__device__ __forceinline__ uint32_t box_row_run(const BrickGrid &bg, const EvalRec &e, const GaussBox &B, float cutoff,
                                                uint32_t r, uint32_t nky, uint32_t &first) {
  const uint32_t dz = r / nky;
  const int kz = (B.zl >> bg.lbz) + (int)dz, ky = (B.yl >> bg.lby) + (int)(r - dz * nky);
  int yl2, yh2, kx0, kx1;
  float xzlo, xzhi;
  if (!slab_part(bg, e, B, cutoff, kz, yl2, yh2, xzlo, xzhi)) return 0u;
  if (ky < (yl2 >> bg.lby) || ky > (yh2 >> bg.lby)) return 0u;
  if (!row_part(bg, e, B, cutoff, ky, yl2, yh2, xzlo, xzhi, kx0, kx1)) return 0u;
  first = (uint32_t)((kz * bg.nby + ky) * bg.nbx + kx0);
  return (uint32_t)(kx1 - kx0 + 1);
}

// Per-lane enumeration: visit(first brick, length, index of the run's first key among the Gaussian's
// keys) for every run; returns the key count.
template <class Visit>
__device__ uint32_t enumerate_bricks(const BrickGrid &bg, const EvalRec &e, const GaussBox &B, float cutoff,
                                     Visit visit) {
  uint32_t count = 0;
  // index ranges are non-negative, so shifts divide by the (power-of-two) brick shape
  for (int kz = B.zl >> bg.lbz; kz <= B.zh >> bg.lbz; ++kz) {
    int yl2, yh2;
    float xzlo, xzhi;
    if (!slab_part(bg, e, B, cutoff, kz, yl2, yh2, xzlo, xzhi)) continue;
    for (int ky = yl2 >> bg.lby; ky <= yh2 >> bg.lby; ++ky) {
      int kx0, kx1;
      if (!row_part(bg, e, B, cutoff, ky, yl2, yh2, xzlo, xzhi, kx0, kx1)) continue;
      const uint32_t row = (uint32_t)((kz * bg.nby + ky) * bg.nbx);
      visit(row + (uint32_t)kx0, (uint32_t)(kx1 - kx0 + 1), count);
      count += (uint32_t)(kx1 - kx0 + 1);
    }
  }
  return count;
}

// Gaussians with more box rows than this are counted by the whole wave, together with the other such
// Gaussians of the wave (a listed box row per lane), instead of by their own lane; the emit pass
// expands them, and those whose runs did not fit the run cache, the same way.
constexpr uint32_t kWaveRows = 16;

// Flattened wave enumeration.  Each lane lists nr rows (the box rows of its Gaussian, or 0); the
// listed rows of the wave are numbered Gaussian by Gaussian in lane order (R: a lane's exclusive
// prefix of nr) and taken 64 at a time, a row per lane.  All shuffles run with every lane active.

__device__ __forceinline__ uint32_t wave_excl_scan_u32(uint32_t v, uint32_t &total) {
  uint32_t incl = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t t = __shfl_up(incl, d, 64);
    if (lane_id() >= d) incl += t;
  }
  total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
  return incl - v;
}

__device__ __forceinline__ float shfl_f(float v, int l) { return __shfl(v, l, 64); }

// The lane listing row q (q below the wave's total): the last lane whose prefix R is <= q.
__device__ __forceinline__ int row_owner(uint32_t q, uint32_t R) {
  int lo = 0, hi = 63;
#pragma unroll
  for (int step = 0; step < 6; ++step) {
    const int mid = (lo + hi + 1) >> 1;
    if ((uint32_t)__shfl((int)R, mid, 64) <= q) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// The geometry of lane o's Gaussian (only what the enumeration reads).
__device__ __forceinline__ void fetch_geometry(const EvalRec &e, const CullRec &c, int o, EvalRec &eb, CullRec &cb) {
  eb.r0 = make_float4(shfl_f(e.r0.x, o), shfl_f(e.r0.y, o), shfl_f(e.r0.z, o), 0.f);
  eb.r1 = make_float4(0.f, 0.f, 0.f, 0.f);
  eb.r2 = eb.r1;
  cb.c0 = make_float4(shfl_f(c.c0.x, o), shfl_f(c.c0.y, o), shfl_f(c.c0.z, o), shfl_f(c.c0.w, o));
  cb.c1 = make_float4(shfl_f(c.c1.x, o), shfl_f(c.c1.y, o), shfl_f(c.c1.z, o), 0.f);
}

// Row item q of the wave's list (valid: q below the total): its owner lane o, and the run of the
// owner's box row q - R_o (0 keys if invalid or the ellipsoid misses the row).
__device__ __forceinline__ uint32_t flat_row_run(const ScanTable &T, float cutoff, const EvalRec &e, const CullRec &c,
                                                 int kscan, uint32_t R, uint32_t q, bool valid, int &o,
                                                 uint32_t &first) {
  o = row_owner(q, R);
  EvalRec eb;
  CullRec cb;
  fetch_geometry(e, c, o, eb, cb);
  const uint32_t Ro = (uint32_t)__shfl((int)R, o, 64);
  const int ko = __shfl(kscan, o, 64);
  first = 0;
  if (!valid) return 0u;
  const BrickGrid &bg = T.s[ko].bg;
  GaussBox B;
  if (!gauss_box(bg, eb, cb, cutoff, B)) return 0u;  // not reached: listed Gaussians have a box
  uint32_t nky;
  box_rows(bg, B, nky);
  return box_row_run(bg, eb, B, cutoff, q - Ro, nky, first);
}

// Run cache: the count pass records each Gaussian's runs (up to kRuns of them, each a 32-bit word
// (first scan-local brick << 4) | (length - 1) for runs of at most 16 bricks starting below 2^28 - 1),
// ended by kRunEnd; a Gaussian whose runs do not fit is marked kRunRedo and the emit pass enumerates
// it again (with the wave).  The emit pass then expands the recorded runs instead of repeating the
// enumeration.  A Gaussian with more than kWaveRows box rows is marked kRunWave instead: it is counted
// and emitted with the wave.
constexpr uint32_t kRunEnd = 0xFFFFFFFFu, kRunRedo = 0xFFFFFFFEu, kRunWave = 0xFFFFFFFDu;

// Fused prep + count: records of Gaussian i (of the concatenated numbering; its parameters are
// entry i - g0 of its scan's arrays), its key count cnt[i], its run cache entry and, per block of
// kPrepThreads Gaussians, the block's key total bsum[block] (the first level of the count scan),
// with bit 63 set if the block holds an invalid Gaussian.
// (register use capped for 6 waves per SIMD: the wave-wide count keeps the records live)
__global__ __launch_bounds__(kPrepThreads) __attribute__((amdgpu_waves_per_eu(6))) void k_prep_count(
    const ScanTable T, float cutoff,
                                                             EvalRec *__restrict__ er, CullRec *__restrict__ cr,
                                                             uint32_t *__restrict__ cnt, uint32_t *__restrict__ runs,
uint64_t *__restrict__ bsum, uint32_t *__restrict__ hist, int64_t hist_len,
    uint32_t *__restrict__ brick_se, int64_t se_len, uint4 *__restrict__ gbox) {
  __shared__ uint64_t wsum[kPrepThreads / 64];
  __shared__ int sbad;
  const int64_t i = (int64_t)blockIdx.x * kPrepThreads + threadIdx.x;
  // the first radix pass's histogram is accumulated by the emit kernel: clear it here
  for (int64_t k = i; k < hist_len; k += (int64_t)gridDim.x * kPrepThreads) hist[k] = 0u;
  // brick list bounds start as (2^32 - 1, 0), which the last sort pass lowers and raises with atomic
  // min / max; bricks without keys keep them (start > end: an empty list)
  for (int64_t k = i; k < se_len; k += (int64_t)gridDim.x * kPrepThreads) brick_se[k] = (k & 1) ? 0u : 0xFFFFFFFFu;
  if (threadIdx.x == 0) sbad = 0;
  __syncthreads();
  __shared__ uint32_t wcount[kPrepThreads];  // key counts of the wide Gaussians, by lane
  uint32_t c = 0, wide_rows = 0;
  bool wide = false;
  int kscan = 0;
  EvalRec e = {};
  CullRec r = {};
  if (i < T.n_total) {
    kscan = T.of_gauss(i);
    const ScanDesc &sd = T.s[kscan];
    if (!make_records(i - sd.g0, sd.mu, sd.ls, sd.quat, sd.amp, sd.relax, cutoff, e, r)) sbad = 1;
    er[i] = e;
    cr[i] = r;
    // the runs are kept in registers (run k goes to rr[k] by selects: the index is not a constant)
    // and written as 16-byte stores
    uint32_t rr[kRuns];
#pragma unroll
    for (int k = 0; k < kRuns; ++k) rr[k] = kRunEnd;
    int nr = 0;
    bool redo = false;
    GaussBox B;
    uint4 vb = make_uint4(1u, 1u, 1u, 0u);  // empty (xl = 1 > xh = 0)
    if (gauss_box(sd.bg, e, r, cutoff, B)) {
      vb = make_uint4((uint32_t)B.xl | ((uint32_t)B.xh << 16), (uint32_t)B.yl | ((uint32_t)B.yh << 16),
                      (uint32_t)B.zl | ((uint32_t)B.zh << 16), 0u);
      uint32_t nky;
      wide_rows = box_rows(sd.bg, B, nky);
      wide = wide_rows > kWaveRows;
      if (!wide)
        c = enumerate_bricks(sd.bg, e, B, cutoff, [&](uint32_t first, uint32_t len, uint32_t) {
          if (nr < kRuns && len <= 16u && first < 0x0FFFFFFFu) {
            const uint32_t word = (first << 4) | (len - 1u);
#pragma unroll
            for (int k = 0; k < kRuns; ++k) rr[k] = nr == k ? word : rr[k];
            ++nr;
          } else {
            redo = true;
          }
        });
    }
    gbox[i] = vb;
    if (wide) rr[0] = kRunWave;
    else if (redo) rr[0] = kRunRedo;
    uint4 *rc = reinterpret_cast<uint4 *>(runs + (int64_t)kRuns * i);
#pragma unroll
    for (int q = 0; q < kRuns / 4; ++q) rc[q] = make_uint4(rr[4 * q], rr[4 * q + 1], rr[4 * q + 2], rr[4 * q + 3]);
  }
  // the wave's wide Gaussians, counted together: a listed box row per lane, each row's run length
  // added to its owner's LDS counter (integer sums: the order does not matter)
  uint32_t tot;
  const uint32_t R = wave_excl_scan_u32(wide ? wide_rows : 0u, tot);
  if (tot) {
    wcount[threadIdx.x] = 0u;
    for (uint32_t t0 = 0; t0 < tot; t0 += 64) {
      const uint32_t q = t0 + (uint32_t)lane_id();
      int o;
      uint32_t first;
      const uint32_t len = flat_row_run(T, cutoff, e, r, kscan, R, min(q, tot - 1), q < tot, o, first);
      if (len) atomicAdd(&wcount[(threadIdx.x & ~63u) + o], len);
    }
    __builtin_amdgcn_wave_barrier();
    if (wide) c = wcount[threadIdx.x];
  }
  if (i < T.n_total) cnt[i] = c;
  uint64_t v = c;
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_down(v, d, 64);
  if (lane_id() == 0) wsum[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t tot = 0;
    for (int w = 0; w < kPrepThreads / 64; ++w) tot += wsum[w];
    bsum[blockIdx.x] = tot | (sbad ? kBadBlock : 0ull);
  }
}

hipError_t launch_prep_count(const ScanTable &T, float cutoff, void *ws, const WsLayout &L, hipStream_t s) {
  char *b = (char *)ws;
  // at least one block: the kernel also clears the first sort pass's histogram and the brick list
  // bounds, which the later kernels read even when there are no Gaussians
  const int blocks = (int)std::max<int64_t>((T.n_total + kPrepThreads - 1) / kPrepThreads, 1);
  prof_begin(s);
  k_prep_count<<<blocks, kPrepThreads, 0, s>>>(T, cutoff, (EvalRec *)(b + L.evalrec), (CullRec *)(b + L.cullrec),
                                               (uint32_t *)(b + L.off), (uint32_t *)(b + L.runs),
                                               (uint64_t *)(b + L.scan_tmp),
                                               (uint32_t *)(b + L.hist), (int64_t)kRadix * L.sort_blocks,
                                               (uint32_t *)(b + L.brick_se), 2 * L.nbricks, (uint4 *)(b + L.gbox));
  prof_end(s, "prep_count");
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------------
// Second level of the count scan: one block turns the per-block key totals into exclusive block
// offsets (64-bit, in place) and writes the whole status block: the key count K, the overflow flag
// (K > capacity) and the non-finite flag (any block flagged); and off[n] = K.  Each thread scans a
// contiguous segment of the totals.

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t t = __shfl_up(v, d, 64);
    if (lane_id() >= d) v += t;
  }
  return v;
}

__device__ __forceinline__ uint64_t wave_incl_scan64(uint64_t v) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint64_t t = __shfl_up(v, d, 64);
    if (lane_id() >= d) v += t;
  }
  return v;
}

constexpr int kBlockScanThreads = 1024;

// step (fit steps only, else NULL): the scans' Adam step counters advance here, before the step's
// Adam update reads them, unless the keys overflowed the capacity (then the step changes nothing).
__global__ __launch_bounds__(kBlockScanThreads) void k_scan_blocks(uint64_t *__restrict__ bsum, int64_t nb,
                                                                    int64_t n, int64_t cap,
                                                                    uint32_t *__restrict__ off, DevStatus *st,
                                                                    int32_t *__restrict__ step, int ns) {
  __shared__ uint64_t wsum[kBlockScanThreads / 64];
  const int t = threadIdx.x;
  const int64_t per = (nb + kBlockScanThreads - 1) / kBlockScanThreads;
  const int64_t s0 = min((int64_t)t * per, nb), s1 = min(s0 + per, nb);
  uint64_t local = 0;
  int bad = 0;
  for (int64_t k = s0; k < s1; ++k) {
    const uint64_t v = bsum[k];
    bad |= (v & kBadBlock) ? 1 : 0;
    local += v & ~kBadBlock;
  }
  bad = __syncthreads_or(bad);
  const uint64_t incl = wave_incl_scan64(local);
  if (lane_id() == 63) wsum[t >> 6] = incl;
  __syncthreads();
  uint64_t woff = 0, total = 0;
  for (int w = 0; w < kBlockScanThreads / 64; ++w) {
    woff += w < (t >> 6) ? wsum[w] : 0;
    total += wsum[w];
  }
  uint64_t run = woff + incl - local;
  for (int64_t k = s0; k < s1; ++k) {
    const uint64_t v = bsum[k] & ~kBadBlock;
    bsum[k] = run;
    run += v;
  }
  if (t == 0) {
    st->n_keys = (int64_t)total;
    st->overflow = (int64_t)total > cap ? 1 : 0;
    st->nonfinite = bad;
    off[n] = (int64_t)total > cap ? (uint32_t)cap : (uint32_t)total;
  }
  if (step && t < ns && (int64_t)total <= cap) step[t] += 1;
}

hipError_t launch_scan_counts(void *ws, const WsLayout &L, int32_t *step, int ns, hipStream_t s) {
  char *b = (char *)ws;
  const int64_t nb = (L.n + kPrepThreads - 1) / kPrepThreads;
  prof_begin(s);
  k_scan_blocks<<<1, kBlockScanThreads, 0, s>>>((uint64_t *)(b + L.scan_tmp), nb, L.n, L.cap,
                                               (uint32_t *)(b + L.off), (DevStatus *)(b + L.status), step, ns);
  prof_end(s, "scan_counts");
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------------
// Emit: the j-th key of Gaussian i is written at slot off[i] + j, with its scan's global brick id
// (the last level of the count scan is done here: off[i] becomes the Gaussian's first slot).  A
// block's Gaussians own a contiguous slot range; when it fits, the block assembles its keys in LDS
// and writes the range out with consecutive threads on consecutive slots.  Wide Gaussians (kRunWave)
// and those whose runs did not fit the cache are expanded by the whole wave: their box rows are
// listed Gaussian by Gaussian, each lane takes a row, and a wave prefix sum of the rows' run lengths
// places each run among its Gaussian's keys in row order.  The first radix pass's digit counts per
// sort tile come from LDS counters (for a block whose range is not staged, from a second read of the
// range it wrote).

// Keys staged per block: 4096 (32 KB of LDS), or 6144 (48 KB, fewer blocks per CU) when the key
// capacity per block suggests that most blocks would not fit 4096 (long-tailed sets).
constexpr int kEmitStageSmall = 4096, kEmitStageLarge = 6144;


// FUSED (at most kFusedScanBlocks blocks): the count scan's second level is done here too.  bex then
// holds the per-block key totals as the prep kernel wrote them, and every block sums them itself: the
// totals of the blocks before it (its offset), all of them (the key count) and their non-finite
// flags; block 0 writes the status block, off[n] and the step counters as the scan kernel would.
// Otherwise bex holds the scanned block offsets and the status block is already written.
constexpr int kFusedScanBlocks = 2048;
static_assert(kFusedScanBlocks % kPrepThreads == 0, "whole loads per thread");

template <int kEmitStage, bool FUSED>
__global__ __launch_bounds__(kPrepThreads) void k_emit(const ScanTable T, float cutoff,
                                                       const EvalRec *__restrict__ er,
                                                       const CullRec *__restrict__ cr,
                                                       const uint32_t *__restrict__ runs, uint32_t *__restrict__ off,
                                                       const uint64_t *__restrict__ bex, int64_t cap,
                                                       DevStatus *st, uint32_t *__restrict__ key_brick,
                                                       uint32_t *__restrict__ key_gid, uint32_t *__restrict__ hist,
                                                       int ntiles, int32_t *__restrict__ step) {
  __shared__ uint32_t sbrick[kEmitStage], sgid[kEmitStage];
  __shared__ uint32_t wtot[kPrepThreads / 64];
  __shared__ uint64_t fpre[kPrepThreads / 64], ftot[kPrepThreads / 64];
  __shared__ int fbad;
  // digit counts of the sort tiles a staged range meets (a range of kEmitStage keys meets at most
  // kEmitTiles tiles)
  constexpr int kEmitTiles = (kEmitStage + kSortTile - 2) / kSortTile + 1;
  __shared__ uint32_t tcnt[kEmitTiles][kRadix];
  const int64_t n = T.n_total;
  uint64_t blk_off;
  if (FUSED) {
    if (threadIdx.x == 0) fbad = 0;
    __syncthreads();
    // (all of the thread's loads issued at once: at most kFusedScanBlocks / kPrepThreads of them)
    constexpr int kPer = kFusedScanBlocks / kPrepThreads;
    uint64_t vv[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int k = (int)threadIdx.x + q * kPrepThreads;
      vv[q] = k < (int)gridDim.x ? bex[k] : 0ull;
    }
    uint64_t pre = 0, tot = 0;
    int bad = 0;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int k = (int)threadIdx.x + q * kPrepThreads;
      const uint64_t v = vv[q];
      bad |= (v & kBadBlock) ? 1 : 0;
      tot += v & ~kBadBlock;
      pre += k < (int)blockIdx.x ? v & ~kBadBlock : 0ull;
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
      pre += __shfl_down(pre, d, 64);
      tot += __shfl_down(tot, d, 64);
    }
    if (bad) atomicOr(&fbad, 1);
    if (lane_id() == 0) {
      fpre[threadIdx.x >> 6] = pre;
      ftot[threadIdx.x >> 6] = tot;
    }
    __syncthreads();
    pre = 0;
    tot = 0;
#pragma unroll
    for (int w2 = 0; w2 < kPrepThreads / 64; ++w2) {
      pre += fpre[w2];
      tot += ftot[w2];
    }
    const bool over = (int64_t)tot > cap;
    if (blockIdx.x == 0) {
      if (threadIdx.x == 0) {
        st->n_keys = (int64_t)tot;
        st->overflow = over ? 1 : 0;
        st->nonfinite = fbad;
        off[n] = over ? (uint32_t)cap : (uint32_t)tot;
      }
      if (step && (int)threadIdx.x < T.ns && !over) step[threadIdx.x] += 1;
    }
    if (over) return;  // uniform per block
    blk_off = pre;
  } else {
    if (st->overflow) return;
    blk_off = bex[blockIdx.x];
  }
  const int64_t i = (int64_t)blockIdx.x * kPrepThreads + threadIdx.x;
  // off[i] holds the key count of Gaussian i; turn it into its first slot: the block's offset plus
  // the exclusive scan of the counts within the block
  const uint32_t c = i < n ? off[i] : 0u;
  const uint32_t incl = wave_incl_scan(c);
  const int w = threadIdx.x >> 6;
  if (lane_id() == 63) wtot[w] = incl;
  __syncthreads();
  uint32_t woff = 0, btot = 0;
#pragma unroll
  for (int k = 0; k < kPrepThreads / 64; ++k) {
    woff += k < w ? wtot[k] : 0u;
    btot += wtot[k];
  }
  const uint32_t blk0 = (uint32_t)blk_off, blk1 = blk0 + btot;
  const uint32_t base = blk0 + woff + incl - c;
  if (i < n) off[i] = base;
  const bool staged = btot <= (uint32_t)kEmitStage;
  // a run of keys of one Gaussian: to LDS when the block's range is staged, else straight to the slots
  auto put_run = [&](uint32_t slot, uint32_t brick, uint32_t len, uint32_t gid) {
    if (staged) {
      for (uint32_t q = 0; q < len; ++q) {
        sbrick[slot - blk0 + q] = brick + q;
        sgid[slot - blk0 + q] = gid;
      }
    } else {
      for (uint32_t q = 0; q < len; ++q) {
        if ((int64_t)(slot + q) < cap) {
          key_brick[slot + q] = brick + q;
          key_gid[slot + q] = gid;
        }
      }
    }
  };
  // Gaussians listed for the flattened wave enumeration: those marked wide by the count pass and
  // those whose runs did not fit the cache
  uint32_t nlist = 0;
  int kscan = 0;
  EvalRec e = {};
  CullRec cg = {};
  if (i < n) {
    kscan = T.of_gauss(i);
    const ScanDesc &sd = T.s[kscan];
    const uint32_t b0 = (uint32_t)sd.b0;
    const uint4 *rc = reinterpret_cast<const uint4 *>(runs + (int64_t)kRuns * i);
    uint32_t rr[kRuns];
#pragma unroll
    for (int q = 0; q < kRuns / 4; ++q) {
      const uint4 v = rc[q];
      rr[4 * q] = v.x;
      rr[4 * q + 1] = v.y;
      rr[4 * q + 2] = v.z;
      rr[4 * q + 3] = v.w;
    }
    auto visit = [&](uint32_t first, uint32_t len, uint32_t j0) { put_run(base + j0, b0 + first, len, (uint32_t)i); };
    if (rr[0] == kRunWave || rr[0] == kRunRedo) {
      e = er[i];
      cg = cr[i];
      GaussBox B;
      uint32_t nky;
      if (gauss_box(sd.bg, e, cg, cutoff, B)) nlist = box_rows(sd.bg, B, nky);
    } else {
      uint32_t j = 0;
#pragma unroll
      for (int k = 0; k < kRuns; ++k) {
        if (rr[k] == kRunEnd) break;
        const uint32_t len = (rr[k] & 15u) + 1u;
        visit(rr[k] >> 4, len, j);
        j += len;
      }
    }
  }
  // the listed Gaussians' keys, a box row per lane: within a 64-row batch an inclusive scan of the
  // run lengths gives each run's place among its owner's keys of the batch; `done` (kept by the
  // owner lane) counts the owner's keys of the earlier batches
  uint32_t tot;
  const uint32_t R = wave_excl_scan_u32(nlist, tot);
  uint32_t done = 0;
  for (uint32_t t0 = 0; t0 < tot; t0 += 64) {
    const uint32_t q = t0 + (uint32_t)lane_id();
    int o;
    uint32_t first;
    const uint32_t len = flat_row_run(T, cutoff, e, cg, kscan, R, min(q, tot - 1), q < tot, o, first);
    uint32_t btot;
    const uint32_t ex = wave_excl_scan_u32(len, btot);
    const uint32_t Ro = (uint32_t)__shfl((int)R, o, 64);
    const int fo = Ro > t0 ? (int)(Ro - t0) : 0;  // the owner's first lane in this batch
    const uint32_t j0 = (uint32_t)__shfl((int)done, o, 64) + ex - (uint32_t)__shfl((int)ex, fo, 64);
    const uint32_t gbase = (uint32_t)__shfl((int)base, o, 64);
    const uint32_t gi = (uint32_t)__shfl((int)(uint32_t)i, o, 64);
    const uint32_t b0 = (uint32_t)T.s[__shfl(kscan, o, 64)].b0;
    if (len) put_run(gbase + j0, b0 + first, len, gi);
    // this lane's own Gaussian: its keys in this batch are those of lanes [a, b)
    const int a = (int)min(R > t0 ? R - t0 : 0u, 64u), b = (int)min(R + nlist > t0 ? R + nlist - t0 : 0u, 64u);
    const uint32_t eb = (uint32_t)__shfl((int)(ex + len), max(b - 1, 0), 64);
    const uint32_t ea = (uint32_t)__shfl((int)ex, min(a, 63), 64);
    done += b > a ? eb - ea : 0u;
  }
  __syncthreads();
  const uint32_t tile0 = blk0 / kSortTile;
  if (staged) {
#pragma unroll
    for (int q = 0; q < kEmitTiles; ++q) tcnt[q][threadIdx.x] = 0u;
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < blk1 - blk0; k += kPrepThreads) {
      const int64_t slot = (int64_t)blk0 + k;
      if (slot < cap) {
        const uint32_t key = sbrick[k];
        key_brick[slot] = key;
        key_gid[slot] = sgid[k];
        atomicAdd(&tcnt[(uint32_t)(slot / kSortTile) - tile0][key & (kRadix - 1)], 1u);
      }
    }
    __syncthreads();
    // integer sums: the histogram does not depend on the order of the additions
    for (int q = 0; q < kEmitTiles; ++q) {
      const uint32_t cq = tcnt[q][threadIdx.x];
      if (cq) atomicAdd(&hist[(int64_t)threadIdx.x * ntiles + tile0 + q], cq);
    }
    return;
  }
  // not staged: the block's keys are in global memory (written by this block's threads before the
  // barrier); count their digits tile by tile
  const uint32_t end = (uint32_t)min((int64_t)blk1, cap);
  for (uint32_t t0 = tile0 * (uint32_t)kSortTile; t0 < end; t0 += (uint32_t)kSortTile) {
    tcnt[0][threadIdx.x] = 0u;
    __syncthreads();
    const uint32_t lo = max(t0, blk0), hi = min(t0 + (uint32_t)kSortTile, end);
    for (uint32_t k = lo + threadIdx.x; k < hi; k += kPrepThreads) atomicAdd(&tcnt[0][key_brick[k] & (kRadix - 1)], 1u);
    __syncthreads();
    const uint32_t cq = tcnt[0][threadIdx.x];
    if (cq) atomicAdd(&hist[(int64_t)threadIdx.x * ntiles + t0 / kSortTile], cq);
    __syncthreads();
  }
}

bool emit_scans(int64_t n) { return n > 0 && (n + kPrepThreads - 1) / kPrepThreads <= kFusedScanBlocks; }

hipError_t launch_emit(const ScanTable &T, float cutoff, uint32_t flags, void *ws, const WsLayout &L, int32_t *step,
                       hipStream_t s) {
  if (T.n_total == 0) return hipSuccess;
  char *b = (char *)ws;
  const int blocks = (int)((T.n_total + kPrepThreads - 1) / kPrepThreads);
  const bool fused = emit_scans(T.n_total);
  // the capacity is sized from the exact key count (times a headroom): its share per block tells
  // whether blocks typically hold more keys than the small stage (the results do not depend on it)
  const bool large = (flags & GS_FLAG_EMIT_STAGE_6K) ||
                     (!(flags & GS_FLAG_EMIT_STAGE_4K) && L.cap / blocks > (int64_t)(7 * kEmitStageSmall / 8));
  auto emit = large ? (fused ? k_emit<kEmitStageLarge, true> : k_emit<kEmitStageLarge, false>)
                     : (fused ? k_emit<kEmitStageSmall, true> : k_emit<kEmitStageSmall, false>);
  prof_begin(s);
  emit<<<blocks, kPrepThreads, 0, s>>>(T, cutoff, (const EvalRec *)(b + L.evalrec), (const CullRec *)(b + L.cullrec),
                                       (const uint32_t *)(b + L.runs), (uint32_t *)(b + L.off),
                                       (const uint64_t *)(b + L.scan_tmp), L.cap, (DevStatus *)(b + L.status),
                                       (uint32_t *)(b + L.key_brick), (uint32_t *)(b + L.key_gid),
                                       (uint32_t *)(b + L.hist), L.sort_blocks, step);
  prof_end(s, "emit");
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------------
// LSD radix sort of (brick id, slot) pairs, 8 bits per pass, stable.  Tiles of 4096 keys.
//   hist:    per-tile digit counts, digit-major [256][tiles] (for the first pass accumulated by the
//            emit kernel); colscan: scanned along the tiles per digit, plus the digit totals.
//   scatter: each wave ranks its 1024 consecutive keys in 16 rounds of 64 (rank among equal digits =
//            wave ballots + a per-wave running count), the four waves' counts are combined into
//            per-digit tile offsets, the tile is reordered by digit in LDS and written out in
//            order, so consecutive threads store consecutive positions of a digit's run.  The last
//            pass writes the Gaussian index of each key (looked up by slot) and the slot, and in
//            place of the sorted brick ids each brick's list bounds (§3.3 per-brick lists).

__device__ __forceinline__ int64_t live_keys(const DevStatus *st, int64_t cap) {
  return st->overflow ? 0 : (st->n_keys < cap ? st->n_keys : cap);
}

__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint32_t *__restrict__ keys, const DevStatus *st,
                                                              int64_t cap, int shift, uint32_t *__restrict__ hist,
                                                              int ntiles) {
  __shared__ uint32_t cnt[kRadix];
  const int t = threadIdx.x;
  cnt[t] = 0;
  __syncthreads();
  const int64_t K = live_keys(st, cap);
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  // thread t counts the tile's keys 16 t .. 16 t + 15 as runs of equal digits: after the previous
  // passes neighbouring keys mostly share this digit, and one LDS atomic per run instead of one per
  // key avoids the lanes of a wave queueing on the same counter
  static_assert(kSortItems == 16, "the histogram reads 16 consecutive keys per thread");
  const int64_t k0 = base + (int64_t)kSortItems * t;
  const int nv = (int)max((int64_t)0, min((int64_t)kSortItems, K - k0));
  if (nv > 0) {
    uint32_t kv[kSortItems];
    if (nv == kSortItems) {
      const uint4 *q = reinterpret_cast<const uint4 *>(keys + k0);  // 64-B aligned
#pragma unroll
      for (int j = 0; j < kSortItems / 4; ++j) {
        const uint4 v = q[j];
        kv[4 * j] = v.x;
        kv[4 * j + 1] = v.y;
        kv[4 * j + 2] = v.z;
        kv[4 * j + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int j = 0; j < kSortItems; ++j) kv[j] = keys[k0 + min(j, nv - 1)];
    }
    uint32_t prev = (kv[0] >> shift) & (kRadix - 1), run = 1;
#pragma unroll
    for (int j = 1; j < kSortItems; ++j) {
      if (j < nv) {
        const uint32_t d = (kv[j] >> shift) & (kRadix - 1);
        if (d != prev) {
          atomicAdd(&cnt[prev], run);
          prev = d;
          run = 0;
        }
        ++run;
      }
    }
    atomicAdd(&cnt[prev], run);
  }
  __syncthreads();
  hist[(int64_t)t * ntiles + blockIdx.x] = cnt[t];
}

// Per digit (one block each): exclusive scan of the digit's tile counts along the tiles, in place,
// and the digit's total.  Thread t owns a contiguous segment of the row (its loads issued eight at a
// time); one block-wide scan of the segment sums gives each segment's start.  The digits' own
// offsets (an exclusive scan of the 256 totals) are formed by every scatter block from the totals.
__global__ __launch_bounds__(kSortThreads) void k_radix_colscan(uint32_t *__restrict__ hist, int ntiles,
                                                                 uint32_t *__restrict__ dtot) {
  __shared__ uint32_t wsum[kSortThreads / 64];
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  uint32_t *row = hist + (int64_t)blockIdx.x * ntiles;
  const int m = (ntiles + kSortThreads - 1) / kSortThreads;
  const int lo = min(t * m, ntiles), hi = min(lo + m, ntiles);
  constexpr int G = 8;
  uint32_t s = 0;
  for (int j0 = lo; j0 < hi; j0 += G) {
    uint32_t v[G];
#pragma unroll
    for (int k = 0; k < G; ++k) v[k] = row[min(j0 + k, hi - 1)];
#pragma unroll
    for (int k = 0; k < G; ++k) s += j0 + k < hi ? v[k] : 0u;
  }
  uint32_t incl = s;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t o = __shfl_up(incl, d, 64);
    if (l >= d) incl += o;
  }
  if (l == 63) wsum[w] = incl;
  __syncthreads();
  uint32_t run = incl - s, tot = 0;
#pragma unroll
  for (int k = 0; k < kSortThreads / 64; ++k) {
    run += k < w ? wsum[k] : 0u;
    tot += wsum[k];
  }
  for (int j0 = lo; j0 < hi; j0 += G) {
    uint32_t v[G];
#pragma unroll
    for (int k = 0; k < G; ++k) v[k] = row[min(j0 + k, hi - 1)];
#pragma unroll
    for (int k = 0; k < G; ++k) {
      if (j0 + k < hi) {
        row[j0 + k] = run;
        run += v[k];
      }
    }
  }
  if (t == 0) dtot[blockIdx.x] = tot;
}

template <bool LAST>
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint32_t *__restrict__ kout,
    uint32_t *__restrict__ vout, const uint32_t *__restrict__ key_gid, uint32_t *__restrict__ gout,
    const DevStatus *st, int64_t cap, int shift, const uint32_t *__restrict__ offsets, int ntiles,
    const uint32_t *__restrict__ dtot, uint32_t *__restrict__ brick_se) {
  __shared__ uint32_t wcnt[kSortThreads / 64][kRadix];  // per-wave running counts, then per-wave offsets
  __shared__ uint32_t tdo[kRadix];                      // digit offsets within the tile
  __shared__ uint32_t goff[kRadix];                     // global offset of the tile's first key of each digit
  __shared__ uint32_t skey[kSortTile], sval[kSortTile];
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const int64_t K = live_keys(st, cap);
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  if (base >= K) return;  // uniform per block
  const int n_tile = (int)min((int64_t)kSortTile, K - base);
  // all of the thread's loads (its keys, its digit's tile offset, the digit totals) are issued first,
  // so the tile pays one memory latency (the ranking's LDS accesses would otherwise hold each key's
  // load until the previous key is ranked)
  // (loads unconditional, at positions clamped to the tile's last key; lanes past the end are masked
  // in the ranking)
  const uint64_t lt = lanemask_lt();
  const int tw = w * (64 * kSortItems) + l;  // position in the tile of the thread's first key
  uint32_t keys[kSortItems], vals[kSortItems], rank[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) keys[r] = kin[base + min(tw + r * 64, n_tile - 1)];
  if (vin) {
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) vals[r] = vin[base + min(tw + r * 64, n_tile - 1)];
  } else {
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) vals[r] = (uint32_t)(base + tw + r * 64);
  }
  const uint32_t toff = offsets[(int64_t)t * ntiles + blockIdx.x];
#pragma unroll
  for (int v = 0; v < kSortThreads / 64; ++v) wcnt[v][t] = 0;
  {  // digit base = exclusive scan of the digit totals (one wave, 4 digits per lane)
    if (t < 64) {
      const uint32_t a0 = dtot[4 * t], a1 = dtot[4 * t + 1], a2 = dtot[4 * t + 2], a3 = dtot[4 * t + 3];
      const uint32_t s4 = a0 + a1 + a2 + a3;
      uint32_t incl = s4;
#pragma unroll
      for (int dd = 1; dd < 64; dd <<= 1) {
        const uint32_t o = __shfl_up(incl, dd, 64);
        if (l >= dd) incl += o;
      }
      const uint32_t ex = incl - s4;
      tdo[4 * t] = ex;
      tdo[4 * t + 1] = ex + a0;
      tdo[4 * t + 2] = ex + a0 + a1;
      tdo[4 * t + 3] = ex + a0 + a1 + a2;
    }
    __syncthreads();
    goff[t] = tdo[t] + toff;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const bool valid = tw + r * 64 < n_tile;  // position in the tile, wave-contiguous
    const uint32_t key = keys[r];
    const uint32_t d = (key >> shift) & (kRadix - 1);
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < kRadixBits; ++bit) {
      const uint64_t bb = __ballot((d >> bit) & 1u);
      m &= ((d >> bit) & 1u) ? bb : ~bb;
    }
    const uint32_t before = (uint32_t)__popcll(m & lt);
    // the running count is shared by the lanes of this wave only; a wave's LDS accesses complete in
    // program order, so every lane reads the count before the group's first lane updates it
    volatile uint32_t *wc = &wcnt[w][0];
    const uint32_t prev = valid ? wc[d] : 0u;
    __builtin_amdgcn_wave_barrier();
    if (valid && before == 0) wc[d] = prev + (uint32_t)__popcll(m);
    __builtin_amdgcn_wave_barrier();
    rank[r] = valid ? prev + before : 0xFFFFFFFFu;
  }
  __syncthreads();
  // per digit: totals over the waves -> exclusive offsets of the waves, and the tile's digit count
  {
    const uint32_t c0 = wcnt[0][t], c1 = wcnt[1][t], c2 = wcnt[2][t], c3 = wcnt[3][t];
    wcnt[0][t] = 0;
    wcnt[1][t] = c0;
    wcnt[2][t] = c0 + c1;
    wcnt[3][t] = c0 + c1 + c2;
    tdo[t] = c0 + c1 + c2 + c3;  // count; scanned below
  }
  __syncthreads();
  if (t < 64) {  // exclusive scan of the 256 digit counts by one wave (4 per lane)
    uint32_t a0 = tdo[4 * t], a1 = tdo[4 * t + 1], a2 = tdo[4 * t + 2], a3 = tdo[4 * t + 3];
    const uint32_t s4 = a0 + a1 + a2 + a3;
    uint32_t incl = s4;
#pragma unroll
    for (int dd = 1; dd < 64; dd <<= 1) {
      const uint32_t o = __shfl_up(incl, dd, 64);
      if (l >= dd) incl += o;
    }
    const uint32_t ex = incl - s4;
    tdo[4 * t] = ex;
    tdo[4 * t + 1] = ex + a0;
    tdo[4 * t + 2] = ex + a0 + a1;
    tdo[4 * t + 3] = ex + a0 + a1 + a2;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    if (rank[r] != 0xFFFFFFFFu) {
      const uint32_t d = (keys[r] >> shift) & (kRadix - 1);
      const uint32_t pos = tdo[d] + wcnt[w][d] + rank[r];
      skey[pos] = keys[r];
      sval[pos] = vals[r];
    }
  }
  __syncthreads();
  // the tile in digit order: positions t, t + 256, ... per thread; in the last pass every Gaussian-index
  // lookup of the thread is issued before the first store.  The last pass writes no brick ids: the
  // tile is now in brick-id order (its keys came sorted by the lower digits and the reorder is
  // stable), and a run of equal ids goes to consecutive positions, so the run's first and last
  // positions bound its brick's list; a brick's runs in different tiles are adjacent in the output,
  // so the minimum of their starts and the maximum of their ends give the whole list (atomic min and
  // max: the result does not depend on the order of the tiles).
  uint32_t gid[kSortItems];
  if (LAST) {
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) gid[j] = key_gid[sval[min(t + j * kSortThreads, n_tile - 1)]];
  }
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const int i = t + j * kSortThreads;
    if (i < n_tile) {
      const uint32_t key = skey[i], val = sval[i];
      const uint32_t d = (key >> shift) & (kRadix - 1);
      const uint32_t pos = goff[d] + ((uint32_t)i - tdo[d]);
      vout[pos] = val;
      if (LAST) {
        gout[pos] = gid[j];
        if (i == 0 || skey[i - 1] != key) atomicMin(&brick_se[2 * (int64_t)key], pos);
        if (i == n_tile - 1 || skey[i + 1] != key) atomicMax(&brick_se[2 * (int64_t)key + 1], pos + 1u);
      } else {
        kout[pos] = key;
      }
    }
  }
}

hipError_t launch_sort(const ScanTable &T, void *ws, const WsLayout &L, hipStream_t s) {
  char *b = (char *)ws;
  DevStatus *st = (DevStatus *)(b + L.status);
  uint32_t *ka = (uint32_t *)(b + L.key_brick), *kb = (uint32_t *)(b + L.keys_alt);
  uint32_t *va = (uint32_t *)(b + L.vals_a), *vb = (uint32_t *)(b + L.vals_b);
  uint32_t *hist = (uint32_t *)(b + L.hist);
  uint32_t *dtot = (uint32_t *)(b + L.scan_tmp);  // digit totals (the scan scratch is free here)
  const int nt = L.sort_blocks;
  if (nt > 0) {
    const uint32_t *kin = ka, *vin = nullptr;
    for (int p = 0; p < L.sort_passes; ++p) {
      const bool last = p == L.sort_passes - 1;
      uint32_t *kout = (p & 1) ? ka : kb;
      uint32_t *vout = last ? (uint32_t *)(b + L.list_slot) : ((p & 1) ? vb : va);
      if (p > 0) {  // the first pass's histogram was accumulated while the keys were emitted
        prof_begin(s);
        k_radix_hist<<<nt, kSortThreads, 0, s>>>(kin, st, L.cap, p * kRadixBits, hist, nt);
        prof_end(s, "radix_hist");
      }
      prof_begin(s);
      k_radix_colscan<<<kRadix, kSortThreads, 0, s>>>(hist, nt, dtot);
      prof_end(s, "radix_scan");
      prof_begin(s);
      if (last)
        k_radix_scatter<true><<<nt, kSortThreads, 0, s>>>(kin, vin, nullptr, vout, (const uint32_t *)(b + L.key_gid),
                                                          (uint32_t *)(b + L.list_gid), st, L.cap, p * kRadixBits,
                                                          hist, nt, dtot, (uint32_t *)(b + L.brick_se));
      else
        k_radix_scatter<false><<<nt, kSortThreads, 0, s>>>(kin, vin, kout, vout, nullptr, nullptr, st, L.cap,
                                                           p * kRadixBits, hist, nt, dtot, nullptr);
      prof_end(s, "radix_scatter");
      kin = kout;
      vin = vout;
    }
  }
  return hipGetLastError();
}

}  // namespace gs
