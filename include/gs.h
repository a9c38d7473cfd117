/*
 * gs.h — C ABI of the MI355X (gfx950) brick-based Gaussian-to-voxel rasterizer.
 *
 * The library renders a voxel grid from 3D anisotropic Gaussians by normalised aggregation and
 * computes the gradient used by the per-scan fit (paper §3.2–§3.3):
 *
 *   w_i(p) = r_i exp(-1/2 (p - mu_i)^T Sigma_i^{-1} (p - mu_i))  if that Mahalanobis d^2 <= cutoff^2
 *   I(p)   = sum_i A_i w_i(p) / (sum_i w_i(p) + eps)
 *   Sigma_i = R(q_i) diag(exp(2 s_i)) R(q_i)^T
 *
 * (§3.2 Eq. (rendering) and the spatial-weight equation after it; §3.1 for the 12 parameters per
 * Gaussian: position 3, covariance 7 = 3 log-scales + 4 quaternion entries, amplitude 1,
 * relaxation factor 1; §3.3 for the 3-sigma truncation, the brick partition and the two gradient
 * equations.)  The cutoff predicate is per pair (voxel, Gaussian) and inclusive; eps is added to
 * the denominator (also in the gradient).
 *
 * Conventions shared by every call:
 *  - Pointers named d_* or documented as "device" are device pointers (e.g. torch tensors on the
 *    GPU); pointers documented as "host" are host memory.  All floating-point data is FP32.
 *  - The caller owns every buffer, including workspaces; the library allocates no device memory
 *    and keeps no state between calls (the one exception: the static scratch array behind
 *    gs_render_fwd_noalloc, part of the library's code object on each GPU).
 *  - Every call is asynchronous on the given stream (a hipStream_t passed as void*; NULL = the null
 *    stream) unless documented as synchronising.  Host-detectable argument errors are returned at
 *    once; errors detected on the device (non-finite input, key-capacity overflow) are latched in
 *    the workspace's status block and returned by gs_status().
 *  - Volumes are [nz][ny][nx] with x fastest.  Voxel (ix, iy, iz) has its centre at
 *    origin + spacing * (ix, iy, iz) in world units.
 *  - Return value: GS_OK (0) or a negative GS_ERR_* code; gs_last_error() describes the last error
 *    of the calling thread.  Results are defined only when the status is GS_OK.
 */
#ifndef GS_H
#define GS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GS_ABI_VERSION 2
#define GS_MAX_SCANS 16 /* scans per batch */

enum {
  GS_OK = 0,
  GS_ERR_INVALID_ARG = -1, /* null pointer, negative size, non-positive dims or spacing, bad options */
  GS_ERR_CAPACITY = -2,    /* more (brick, Gaussian) keys than the workspace's key capacity */
  GS_ERR_NONFINITE = -3,   /* NaN/Inf parameter, zero quaternion or relaxation factor <= 0 */
  GS_ERR_HIP = -4,         /* a HIP runtime call failed */
  GS_ERR_UNSUPPORTED = -5  /* valid but not supported by this library (e.g. a brick shape) */
};

/* Gaussian set (§3.1): n Gaussians, structure of arrays, device pointers. */
typedef struct {
  int64_t n;
  const float *mu;        /* [n][3] centre, world units */
  const float *log_scale; /* [n][3] natural log of the standard deviation along each principal axis */
  const float *quat;      /* [n][4] rotation (w, x, y, z); any nonzero norm, normalised internally */
  const float *amp;       /* [n]    amplitude A_i */
  const float *relax;     /* [n]    relaxation factor r_i > 0, or NULL meaning r_i = 1 */
} gs_gaussians_t;

/* Output grid (any shape and resolution: rendering at an arbitrary target shape, §4.2).  Each
 * dimension is at most 65535 voxels (GS_ERR_UNSUPPORTED beyond). */
typedef struct {
  int32_t nx, ny, nz;
  float origin[3];  /* centre of voxel (0,0,0) */
  float spacing[3]; /* > 0 */
} gs_grid_t;

/* opts.flags bits */
#define GS_FLAG_FORWARD_ONLY 1u /* workspace without the backward's partial sums (48 B per key less);
                                   the backward and the fit reject such options */
/* Tuning bits: they change speed only; every result is bitwise the same with or without them. */
#define GS_FLAG_BWD_ONE_BRICK (1u << 4)  /* backward: one brick per one-wave workgroup (default: eight
                                            consecutive bricks whose keys are ordered together, per
                                            eight-wave workgroup) */
#define GS_FLAG_BWD_TWO_BRICKS (1u << 8) /* backward: two consecutive bricks per one-wave workgroup (not
                                            with GS_FLAG_BWD_ONE_BRICK) */
#define GS_FLAG_BWD_WINDOW_256 (1u << 5) /* backward: keys ordered in windows of half the default size
                                            (default: 2048 keys for eight bricks, 512 for one or two) */
#define GS_FLAG_EMIT_STAGE_4K (1u << 6)  /* key emission stages up to 4096 keys per workgroup in LDS ... */
#define GS_FLAG_EMIT_STAGE_6K (1u << 7)  /* ... or up to 6144 (neither: chosen from the key capacity per
                                            workgroup; not both) */

/* Rasterizer options.  Brick shape (bx, by, bz) in voxels (§3.3 uses 8x8x4; the library also runs
 * 4x8x4 and 16x8x4, a choice that changes speed and FP32 summation order only);
 * gs_brick_supported() tells.  cutoff: Mahalanobis truncation radius (3 = the 3-sigma ellipsoid).
 * eps: denominator regulariser, > 0 (the rendering equation has none; with eps = 0 a voxel that no
 * Gaussian reaches would be 0/0, so the library requires a positive eps). */
typedef struct {
  int32_t bx, by, bz;
  float cutoff;
  float eps;
  uint32_t flags; /* GS_FLAG_* bits; the same flags must be used for sizing and for every call */
} gs_opts_t;

/* Binning workspace: caller-owned device memory of gs_workspace_size() bytes for `key_capacity`
 * (brick, Gaussian) keys.  Holds the per-Gaussian records, the brick-sorted key lists, the brick
 * offsets, the backward's per-key partial sums and the status block.  One workspace serves one
 * Gaussian set and grid (or one batch of scans) at a time. */
typedef struct {
  void *ws;
  size_t ws_bytes;
  int64_t key_capacity;
} gs_bins_t;

/* Gradient outputs (device, written, not accumulated).  Any pointer may be NULL to skip it. */
typedef struct {
  float *d_mu;        /* [n][3] */
  float *d_log_scale; /* [n][3] */
  float *d_quat;      /* [n][4] gradient w.r.t. the raw (unnormalised) quaternion */
  float *d_amp;       /* [n] */
  float *d_relax;     /* [n] (ignored when the Gaussians have relax == NULL) */
} gs_grads_t;

/* Adam hyper-parameters; lr per parameter group in the order mu, log_scale, quat, amp, relax. */
typedef struct {
  float lr[5];
  float beta1, beta2, eps;
} gs_adam_t;

/* Fit state: parameters updated in place, Adam moments and the device step counter. */
typedef struct {
  int64_t n;
  float *mu, *log_scale, *quat, *amp; /* device, [n][3], [n][3], [n][4], [n] */
  float *relax;                        /* device [n], or NULL (r = 1, not optimised) */
  float *m, *v;    /* device [12 n] each: groups mu (3n), log_scale (3n), quat (4n), amp (n), relax (n) */
  int32_t *step;   /* device: Adam steps taken so far (0 before the first step); one counter per scan
                      of a batch ([ns]), a scalar for the single-scan calls */
} gs_fit_state_t;

/* Per-step fit options: HR grid, rasterizer options, z-downsampling factor of the LR observation
 * (LR slice k = mean of HR slices f*k .. f*k+f-1) and Adam. */
typedef struct {
  gs_grid_t hr;
  gs_opts_t opts;
  int32_t zdown;
  int32_t loss; /* 0 = L1 on the z-mean (the only loss of the fit) */
  gs_adam_t adam;
} gs_fit_opts_t;

/* Caller-owned per-step buffers of the fit (device). */
typedef struct {
  float *I, *W;        /* [nz][ny][nx] forward outputs (kept for the backward) */
  float *dL_dI;        /* [nz][ny][nx]; used only when zdown differs from the brick depth bz (else
                          the loss is fused into the backward and this may be NULL) */
  gs_grads_t grads;    /* [n]-sized gradient arrays (written); d_mu, d_log_scale, d_quat, d_amp required */
  void *scratch;       /* >= gs_fit_scratch_bytes(&hr) bytes */
  size_t scratch_bytes;
  float *loss;         /* device: the step's loss, one per scan of a batch ([ns]) */
} gs_fit_buffers_t;

/* A batch of independent scans handled by the same launches (each phase of the method is one launch
 * over the bricks of all scans; §3.3's brick partition applies to each scan's own grid).  Scan k
 * owns the n[k] Gaussians that follow those of scans 0..k-1 in the concatenated Gaussian numbering,
 * and its volumes (I, W, dL_dI: grid[k].nz * ny * nx voxels) and LR observation follow those of
 * scans 0..k-1 in the concatenated arrays.  Results of every scan are bitwise identical to those of
 * the single-scan calls on that scan alone.  The single-scan calls are the ns = 1 case.
 * The Gaussians come either from one concatenated set (the `g` argument of the calls, sets = NULL)
 * or, for gs_bin_query_batch, gs_bin_batch, gs_render_fwd_batch and gs_count_pairs_batch only, from
 * one set per scan (sets[k], with sets[k].n == n[k]; then `g` must be NULL): resident sets are then
 * rendered together without being copied into one array. */
typedef struct {
  int32_t ns;                  /* 1 .. GS_MAX_SCANS */
  const int64_t *n;            /* host [ns]: Gaussians per scan (>= 0) */
  const gs_grid_t *grid;       /* host [ns]: grid per scan */
  const gs_gaussians_t *sets;  /* host [ns] or NULL (see above) */
} gs_batch_t;

/* Device status block (read by gs_status). */
typedef struct {
  int64_t n_keys;     /* exact number of (brick, Gaussian) keys of the last binning */
  int32_t overflow;   /* n_keys > key_capacity: the bins (and everything after) are invalid */
  int32_t nonfinite;  /* some Gaussian had a non-finite parameter, zero quaternion or r <= 0 */
} gs_status_t;

/* ---- sizes and capabilities ---------------------------------------------------------------- */

/* Bytes of binning workspace for n Gaussians on `grid` with `opts` and room for key_capacity keys.
 * Host only; allocates nothing. */
int gs_workspace_size(int64_t n, const gs_grid_t *grid, const gs_opts_t *opts, int64_t key_capacity,
                      size_t *bytes /* host out */);

/* Bytes of scratch for the loss reductions over nvox voxels. */
size_t gs_loss_scratch_bytes(int64_t nvox);

/* Bytes of scratch for gs_fit_step on the HR grid hr (0 for an invalid grid). */
size_t gs_fit_scratch_bytes(const gs_grid_t *hr);

/* Batch forms of the two sizes above (0 for an invalid batch). */
int gs_workspace_size_batch(const gs_batch_t *batch, const gs_opts_t *opts, int64_t key_capacity,
                            size_t *bytes /* host out */);
size_t gs_fit_scratch_bytes_batch(const gs_batch_t *batch);

/* 1 if the brick shape is supported by the kernels of this library, else 0. */
int gs_brick_supported(int32_t bx, int32_t by, int32_t bz);

/* ---- binning (§3.3: for each brick, the Gaussians whose 3-sigma ellipsoid meets it) --------- */

/* Count the (brick, Gaussian) keys of `g` on `grid` and return the exact count in *n_keys (host).
 * Needs a workspace sized for key_capacity >= 0 (0 is enough).  SYNCHRONISES the stream. */
int gs_bin_query(const gs_gaussians_t *g, const gs_grid_t *grid, const gs_opts_t *opts, const gs_bins_t *bins,
                 void *stream, int64_t *n_keys /* host out */);

/* Build the per-brick Gaussian lists: per-Gaussian records, keys (brick id, Gaussian) for every
 * brick that may meet the Gaussian's ellipsoid, radix sort on brick id (stable: ascending Gaussian
 * index within a brick), brick offsets.  Resets the status block.  If the key count exceeds
 * bins->key_capacity, the overflow flag is latched and every later call on these bins leaves its
 * outputs unwritten until the next gs_bin. */
int gs_bin(const gs_gaussians_t *g, const gs_grid_t *grid, const gs_opts_t *opts, const gs_bins_t *bins,
           void *stream);

/* ---- forward (§3.2 Eq. (rendering); §3.3 forward cache) ------------------------------------- */

/* Render I (and the per-voxel weight sum W, the cache the backward reads; may be NULL) on `grid`
 * from bins built by gs_bin with the same g, grid and opts.  I, W: device [nz][ny][nx].  Each
 * voxel's sums run over its Gaussians in ascending index order as four interleaved partial sums
 * added in a fixed order (bitwise deterministic). */
int gs_render_fwd(const gs_gaussians_t *g, const gs_grid_t *grid, const gs_opts_t *opts, const gs_bins_t *bins,
                  float *I, float *W, void *stream);

/* Number of useful pairs (voxel, Gaussian) with d^2 <= cutoff^2, written to *d_count (device
 * int64).  Same bins contract as gs_render_fwd.  For measurement. */
int gs_count_pairs(const gs_gaussians_t *g, const gs_grid_t *grid, const gs_opts_t *opts, const gs_bins_t *bins,
                   int64_t *d_count, void *stream);

/* Evaluation counts of the forward and backward kernels on these bins, for measurement (how much
 * of the work they issue is useful).  d_counts: device int64[6], overwritten:
 *   [0] useful pairs (voxel, Gaussian) with d^2 <= cutoff^2 (as gs_count_pairs);
 *   [1] forward: (voxel, Gaussian) evaluations of real cell-list entries inside the grid;
 *   [2] forward: issued lane-voxel slots (every lane of every list iteration, padding included);
 *   [3] backward: voxel evaluations of the rows that pass the row test (BX per row);
 *   [4] backward: issued lane-voxel slots (64 lanes x BX per row iteration a wave executes);
 *   [5] backward: rows in the keys' voxel boxes.
 * Same bins contract as gs_render_fwd. */
int gs_count_evals(const gs_gaussians_t *g, const gs_grid_t *grid, const gs_opts_t *opts, const gs_bins_t *bins,
                   int64_t *d_counts, void *stream);

/* ---- backward (§3.3 gradient equations) ---------------------------------------------------- */

/* Gradients of a loss L w.r.t. every Gaussian parameter, given the forward's I and W and
 * dL_dI = dL/dI per voxel (all device [nz][ny][nx]).  Per brick, per Gaussian partial sums are
 * written to the workspace (no atomics); a per-Gaussian fixed-order reduction then applies the
 * chain rule to (mu, log_scale, quat, amp, relax).  Bitwise deterministic. */
int gs_render_bwd(const gs_gaussians_t *g, const gs_grid_t *grid, const gs_opts_t *opts, const gs_bins_t *bins,
                  const float *I, const float *W, const float *dL_dI, const gs_grads_t *grads, void *stream);

/* ---- losses of the fit ------------------------------------------------------------------------ */

/* L = mean((I - T)^2) over nvox voxels; dL_dI = 2 (I - T) / nvox.  loss: device scalar. */
int gs_loss_mse(const float *I, const float *T, int64_t nvox, float *dL_dI, float *loss, void *scratch,
                size_t scratch_bytes, void *stream);

/* Fit loss: LR = mean of zdown consecutive z slices of I ([nz/zdown][ny][nx], nz % zdown == 0);
 * L = mean |LR - obs|; dL_dI = sign(LR - obs) / (zdown * nLR) broadcast to the zdown HR slices
 * (sign(0) = 0).  loss: device scalar. */
int gs_loss_l1_zmean(const float *I, const float *obs, const gs_grid_t *hr, int32_t zdown, float *dL_dI, float *loss,
                     void *scratch, size_t scratch_bytes, void *stream);

/* ---- optimiser and fit step ---------------------------------------------------------------- */

/* One Adam step with bias correction on every parameter group of st, from grads (all required
 * except d_relax; groups with lr 0 keep their values).  Increments *st->step. */
int gs_adam_step(const gs_fit_state_t *st, const gs_grads_t *grads, const gs_adam_t *hp, const gs_bins_t *bins,
                 void *stream);

/* One step of the per-scan zero-shot fit (§3.2: the whole rendering is differentiable and optimised
 * end to end; Fig. 1 for the fit loop): bin -> render -> z-mean ->
 * L1 vs lr_obs -> backward -> Adam.  lr_obs: device [hr.nz/zdown][hr.ny][hr.nx].  Writes I, W, the
 * gradients and the loss; updates the parameters, the moments and *step.  The gradient reduction
 * is fused with Adam; when zdown equals the brick depth the loss is also computed inside the
 * backward kernel.  No host synchronisation; check gs_status() for capacity overflow (the step then
 * writes none of its outputs: the parameters, the moments, *step and the loss keep their values). */
int gs_fit_step(const gs_fit_state_t *st, const float *lr_obs, const gs_fit_opts_t *fo, const gs_bins_t *bins,
                const gs_fit_buffers_t *buf, void *stream);

/* ---- batches of scans (many scans of uneven size in one launch per phase) ------------------- */

/* Each call below equals its single-scan namesake applied to every scan of `batch`, with g the
 * concatenated Gaussian set (g->n = sum of batch->n) and every volume argument the concatenation
 * of the scans' volumes in batch order.  One workspace serves the whole batch
 * (gs_workspace_size_batch); keys and bricks of all scans share its capacity. */
int gs_bin_query_batch(const gs_gaussians_t *g, const gs_batch_t *batch, const gs_opts_t *opts,
                       const gs_bins_t *bins, void *stream, int64_t *n_keys /* host out */);
int gs_bin_batch(const gs_gaussians_t *g, const gs_batch_t *batch, const gs_opts_t *opts, const gs_bins_t *bins,
                 void *stream);
int gs_render_fwd_batch(const gs_gaussians_t *g, const gs_batch_t *batch, const gs_opts_t *opts,
                        const gs_bins_t *bins, float *I, float *W, void *stream);
int gs_count_pairs_batch(const gs_gaussians_t *g, const gs_batch_t *batch, const gs_opts_t *opts,
                         const gs_bins_t *bins, int64_t *d_count, void *stream);
int gs_render_bwd_batch(const gs_gaussians_t *g, const gs_batch_t *batch, const gs_opts_t *opts,
                        const gs_bins_t *bins, const float *I, const float *W, const float *dL_dI,
                        const gs_grads_t *grads, void *stream);

/* One fit step of every scan of the batch (as gs_fit_step per scan; fo->hr is not read, the grids
 * come from the batch; every scan's nz must be a multiple of fo->zdown).  st holds the concatenated
 * parameters and moments ([12 n_total] in the group layout over the whole set) and one step counter
 * per scan; lr_obs the concatenated LR observations; buf->loss receives one loss per scan and
 * buf->scratch must hold gs_fit_scratch_bytes_batch(batch) bytes.  Scans may be at different steps
 * (each has its own Adam bias correction). */
int gs_fit_step_batch(const gs_fit_state_t *st, const float *lr_obs, const gs_batch_t *batch,
                      const gs_fit_opts_t *fo, const gs_bins_t *bins, const gs_fit_buffers_t *buf, void *stream);

/* ---- rendering without allocation ------------------------------------------------------------ */

/* Bytes of the static device scratch behind gs_render_fwd_noalloc (64 MiB), held by the library on
 * every GPU it renders on until the process ends. */
#define GS_STATIC_SCRATCH_BYTES (64ull << 20)

/* For callers that cannot allocate device memory or pass a workspace (code under HIP graph
 * capture, serving loops and harnesses that forbid allocation): gs_bin followed by gs_render_fwd
 * (forward-only), with the binning workspace in the library's static scratch instead of a
 * caller-owned one.  I (and W, may be NULL) are caller-owned device [nz][ny][nx] outputs, bitwise
 * equal to those of gs_bin + gs_render_fwd on the same inputs.  Allocates nothing and does not
 * synchronise.  The key capacity is whatever the scratch holds after the per-Gaussian and
 * per-brick parts (about 2.3M keys for 20k Gaussians on 64x64x32); a set whose per-Gaussian and
 * per-brick parts alone exceed GS_STATIC_SCRATCH_BYTES is rejected with GS_ERR_INVALID_ARG before
 * anything is launched.  More keys than the capacity are detected on the device: I and W are then
 * left unwritten and the status says overflow.  d_status (device, may be NULL) receives the
 * binning's status block (key count, overflow, non-finite flags) when the call's work has run.
 * Every call on one GPU shares that GPU's scratch: calls that overlap in time on one GPU (on
 * different streams, or from different threads) race and must be serialised by the caller. */
int gs_render_fwd_noalloc(const gs_gaussians_t *g, const gs_grid_t *grid, const gs_opts_t *opts, float *I, float *W,
                          gs_status_t *d_status, void *stream);

/* ---- status, errors, profiling ---------------------------------------------------------------- */

/* Copy the status block of `bins` to *out (host).  SYNCHRONISES the stream.  Returns GS_OK,
 * GS_ERR_CAPACITY or GS_ERR_NONFINITE according to the latched flags. */
int gs_status(const gs_bins_t *bins, void *stream, gs_status_t *out /* host */);

/* Thread-local description of the last error returned to this thread. */
const char *gs_last_error(void);

/* Kernel timing: when enabled, every kernel the library launches is bracketed by HIP events on
 * the launch stream; gs_profile_read() synchronises, accumulates the elapsed times per kernel name
 * and returns up to `cap` entries (name, launches, total milliseconds) in host arrays. */
int gs_profile_enable(int on);
int gs_profile_read(void *stream, int cap, char (*names)[48], int64_t *launches, double *total_ms,
                    int *n_out);
int gs_profile_reset(void);

#ifdef __cplusplus
}
#endif
#endif /* GS_H */
