// Internal declarations of the gfx950 rasterizer library (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gs.h"

namespace gs {

// log2(e) and the exponent scale: w = r exp(-d^2/2) = exp2(q + log2 r) with q = -1/2 log2(e) d^2.
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kHalfLog2e = 0.7213475204444817f;

// Per-Gaussian evaluation record (48 B), written by the prep kernel and staged through LDS by the
// forward and backward kernels:
//   r0 = (mu_x, mu_y, mu_z, A)
//   r1 = (Q_xx, 2 Q_xy, 2 Q_xz, thr + log2 r)     Q = -1/2 log2(e) Sigma^{-1}, thr = -1/2 log2(e) cutoff^2
//   r2 = (Q_yy, 2 Q_yz, Q_zz, log2 r)
// On a voxel row (fixed y, z) the exponent is q(dx) = Q_xx dx^2 + b dx + c with
// b = 2 Q_xy dy + 2 Q_xz dz and c = Q_yy dy^2 + 2 Q_yz dy dz + Q_zz dz^2 + log2 r (delta = p - mu);
// the pair is kept iff q >= thr + log2 r (i.e. d^2 <= cutoff^2) and w = r exp(-d^2/2) = exp2(q).
struct __align__(16) EvalRec {
  float4 r0, r1, r2;
};

// Per-Gaussian culling record (32 B): covariance entries and a validity flag.
//   c0 = (S_xx, S_yy, S_zz, S_xy), c1 = (S_xz, S_yz, valid ? 1 : 0, 0)
struct __align__(16) CullRec {
  float4 c0, c1;
};

// Device status block at offset 0 of every workspace (layout of gs_status_t + spare).
struct DevStatus {
  int64_t n_keys;
  int32_t overflow;
  int32_t nonfinite;
  int32_t spare[12];
};

// Brick grid geometry of one scan.  Brick shape (bx, 8, 4) with bx in {4, 8, 16}.
struct BrickGrid {
  int nx, ny, nz;    // voxels
  int nbx, nby, nbz; // bricks per axis
  uint8_t lbx, lby, lbz;  // log2 of the brick shape (bricks are powers of two on every axis)
  // n / nbx and n / nby for n < 2^31 as (umulhi(n, m) + n) >> s (multiply-high division by an
  // invariant divisor, constants from the host), so that a workgroup's brick coordinates need no
  // vector instructions
  uint8_t sbx, sby;
  uint32_t mbx, mby;
  int64_t nbricks;
  float ox, oy, oz;  // origin
  float hx, hy, hz;  // spacing
  float ihx, ihy, ihz;  // 1 / spacing
};

// Several scans (each its own grid and Gaussian set) are processed by the same launches: their
// Gaussians, bricks, volumes and observations are concatenated, and every kernel finds its scan in a
// small table passed by value as a kernel argument.  A single scan is the one-entry table.
constexpr int kMaxScans = 16;

// Bricks per backward workgroup (consecutive bricks of a scan whose keys are ordered together): 8
// (eight waves), or 2 or 1 (one wave) with GS_FLAG_BWD_TWO_BRICKS or GS_FLAG_BWD_ONE_BRICK.
__host__ __device__ inline int bwd_bricks_of(uint32_t flags) {
  return (flags & GS_FLAG_BWD_ONE_BRICK) ? 1 : (flags & GS_FLAG_BWD_TWO_BRICKS) ? 2 : 8;
}

struct ScanDesc {
  BrickGrid bg;
  // the scan's own Gaussian parameters (n entries each; relax may be NULL); for a concatenated set
  // these point into it at Gaussian g0
  const float *mu, *ls, *quat, *amp, *relax;
  int64_t g0, n;  // Gaussians [g0, g0 + n) of the concatenated numbering
  int64_t b0;     // first (global) brick of the scan
  int64_t p0;     // first (global) brick group of the scan (the backward takes bwd_bricks bricks per workgroup)
  int64_t v0;     // first voxel of the scan's volume in the concatenated volumes
  int64_t o0;     // first LR voxel of the scan's observation in the concatenated observations
  float gscale;   // fit loss: dL/dI magnitude 1 / (zdown * nLR)
  float lscale;   // fit loss: 1 / nLR
};

struct ScanTable {
  int32_t ns;
  int32_t bwd_bricks;  // bricks per backward group (bwd_bricks_of the options' flags)
  int64_t n_total, nbricks_total, ngroups_total;
  ScanDesc s[kMaxScans];
  __host__ __device__ __forceinline__ int of_gauss(int64_t i) const {
    int k = 0;
    while (k + 1 < ns && i >= s[k + 1].g0) ++k;
    return k;
  }
  __host__ __device__ __forceinline__ int of_brick(int64_t b) const {
    int k = 0;
    while (k + 1 < ns && b >= s[k + 1].b0) ++k;
    return k;
  }
  __host__ __device__ __forceinline__ int of_group(int64_t q) const {
    int k = 0;
    while (k + 1 < ns && q >= s[k + 1].p0) ++k;
    return k;
  }
};

// the table travels by value as a kernel argument (at most 4 KB of arguments per launch)
static_assert(sizeof(ScanTable) <= 3072, "scan table too large for a kernel argument");

// Radix sort tiling.
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;

// Gaussians per prep / emit block: the first level of the key-count scan.  A block's key total
// carries kBadBlock when the block holds an invalid Gaussian (non-finite parameter, zero quaternion
// or r <= 0).
constexpr int kPrepThreads = 256;
constexpr int kRuns = 8;  // brick runs cached per Gaussian between the count and the emit pass
// Voxel box of a Gaussian (its padded 3-sigma extent in voxel indices), written by the prep kernel for
// the backward's ordering pass: uint4 (xl | xh << 16, yl | yh << 16, zl | zh << 16, 0), empty
// (xl > xh) for a Gaussian without keys.  16-bit indices: grid dimensions are at most kMaxGridDim.
constexpr int kMaxGridDim = 65535;
static_assert(kRuns % 4 == 0, "the run cache is read and written as 16-byte words");
constexpr uint64_t kBadBlock = 1ull << 63;

// Workspace layout, all offsets in bytes from the workspace base, 256-B aligned.
//   gbox: uint4 [n] voxel boxes (see kMaxGridDim).
//   off: uint32 [n + 1]: key counts per Gaussian, after the emit the first key slot of each
//        Gaussian (keys are numbered Gaussian-major); off[n] = the key count.
//   scan_tmp: per-block key totals of the count scan (uint64), later the radix digit totals.
//   key_brick, key_gid: uint32 [cap] keys in slot order; keys_alt, vals_a, vals_b: radix ping-pong.
//   list_gid, list_slot: uint32 [cap] the keys sorted by brick: Gaussian index and key slot.
//   brick_se: uint32 [B][2] each brick's list bounds (first position, end) in the sorted keys,
//   (2^32 - 1, 0) for a brick without keys (any start >= end is an empty list).  partials: 48 B per key slot (backward; absent in a forward-only
//   workspace).
struct WsLayout {
  int64_t n = 0, cap = 0, nbricks = 0;
  int sort_blocks = 0;  // tiles per radix pass (covers cap keys)
  int sort_passes = 0;  // ceil(bits(nbricks) / 8), at least 1
  size_t status = 0, evalrec = 0, cullrec = 0, off = 0, runs = 0, gbox = 0, key_brick = 0, key_gid = 0, keys_alt = 0, vals_a = 0,
         vals_b = 0, list_gid = 0, list_slot = 0, brick_se = 0, hist = 0, scan_tmp = 0, partials = 0, total = 0;
};

// Host-side helpers (api.cpp).
bool make_brick_grid(const gs_grid_t *grid, const gs_opts_t *opts, BrickGrid *bg);
WsLayout make_layout(int64_t n, int64_t nbricks, int64_t cap, bool partials);

// Launch bookkeeping for the optional kernel timing (api.cpp).
void prof_begin(hipStream_t s);
void prof_end(hipStream_t s, const char *name);

// Kernel launchers (bin.hip, render.hip, reduce.hip, fit.hip).  Return hipGetLastError() of the
// launches.  `g` / `st` hold the concatenated Gaussians of all scans of T.
hipError_t launch_prep_count(const ScanTable &T, float cutoff, void *ws, const WsLayout &L, hipStream_t s);
hipError_t launch_scan_counts(void *ws, const WsLayout &L, int32_t *step, int ns, hipStream_t s);
// emit_scans(n): the emit does the count scan's second level itself (a one-block scan kernel is then
// not launched); step as for launch_scan_counts.
bool emit_scans(int64_t n);
hipError_t launch_emit(const ScanTable &T, float cutoff, uint32_t flags, void *ws, const WsLayout &L, int32_t *step,
                       hipStream_t s);
hipError_t launch_sort(const ScanTable &T, void *ws, const WsLayout &L, hipStream_t s);
hipError_t launch_fwd(const ScanTable &T, int bx, float cutoff, float eps, const void *ws, const WsLayout &L,
                      float *I, float *W, hipStream_t s);
hipError_t launch_count_pairs(const ScanTable &T, int bx, float cutoff, const void *ws, const WsLayout &L,
                              int64_t *d_count, hipStream_t s);
// Evaluation counts (gs_count_evals): kEvalCounts int64 entries.
constexpr int kEvalCounts = 6;
hipError_t launch_count_evals(const ScanTable &T, int bx, uint32_t flags, float cutoff, const void *ws,
                              const WsLayout &L, int64_t *d_counts, hipStream_t s);
hipError_t launch_bwd(const ScanTable &T, int bx, uint32_t flags, float cutoff, float eps, void *ws, const WsLayout &L,
                      const float *I, const float *W, const float *dLdI, hipStream_t s);
hipError_t launch_bwd_fit(const ScanTable &T, int bx, uint32_t flags, float cutoff, float eps, void *ws,
                          const WsLayout &L, const float *I, const float *W, const float *obs, float *loss_part,
                          hipStream_t s);
hipError_t launch_reduce_chain(const gs_gaussians_t &g, const void *ws, const WsLayout &L, const gs_grads_t &gr,
                               hipStream_t s);
hipError_t launch_reduce_adam(const ScanTable &T, const gs_fit_state_t &g, const void *ws, const WsLayout &L,
                              const gs_grads_t &gr, const gs_adam_t &hp, const float *loss_part, float *loss,
                              hipStream_t s);
hipError_t launch_loss_mse(const float *I, const float *T, int64_t nvox, float *g, float *loss, void *scratch,
                           hipStream_t s);
hipError_t launch_loss_l1z(const float *I, const float *obs, int nx, int ny, int nz, int f, float *g, float *loss,
                           void *scratch, hipStream_t s, const DevStatus *st = nullptr);
hipError_t launch_adam(const gs_fit_state_t &st, const gs_grads_t &gr, const gs_adam_t &hp, const void *ws_status,
                       hipStream_t s);

// Loss reduction tiling.
constexpr int kLossThreads = 256;
constexpr int kLossItems = 16;
int loss_blocks(int64_t nvox);

}  // namespace gs
