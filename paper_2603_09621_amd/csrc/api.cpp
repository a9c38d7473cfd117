// C ABI of the rasterizer library: argument checks, workspace layout, launch sequences, status,
// errors and optional kernel timing.  Declared in include/gs.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "gs_internal.h"

namespace gs {

static thread_local std::string g_last_error;

static int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
static int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

static int hip_fail(hipError_t e, const char *where) {
  return fail(GS_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

// ---- optional kernel timing ---------------------------------------------------------------------

struct ProfRec {
  std::string name;
  hipEvent_t a, b;
};
static std::mutex g_prof_mu;
static bool g_prof_on = false;
static std::vector<ProfRec> g_prof_pending;
static std::vector<hipEvent_t> g_prof_pool;
static std::vector<std::pair<std::string, std::pair<int64_t, double>>> g_prof_acc;
static thread_local hipEvent_t g_prof_open = nullptr;

static hipEvent_t prof_event() {
  if (!g_prof_pool.empty()) {
    hipEvent_t e = g_prof_pool.back();
    g_prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void prof_begin(hipStream_t s) {
  if (!g_prof_on) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_open = prof_event();
  if (g_prof_open) (void)hipEventRecord(g_prof_open, s);
}

void prof_end(hipStream_t s, const char *name) {
  if (!g_prof_on || !g_prof_open) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  hipEvent_t e = prof_event();
  if (!e) return;
  (void)hipEventRecord(e, s);
  g_prof_pending.push_back(ProfRec{name, g_prof_open, e});
  g_prof_open = nullptr;
}

// ---- geometry and workspace layout ---------------------------------------------------------------

static bool brick_supported(int bx, int by, int bz) { return (bx == 4 || bx == 8 || bx == 16) && by == 8 && bz == 4; }

bool make_brick_grid(const gs_grid_t *grid, const gs_opts_t *opts, BrickGrid *bg) {
  bg->nx = grid->nx;
  bg->ny = grid->ny;
  bg->nz = grid->nz;
  auto ilog2 = [](int v) {
    int l = 0;
    while ((1 << (l + 1)) <= v) ++l;
    return l;
  };
  bg->lbx = ilog2(opts->bx);
  bg->lby = ilog2(opts->by);
  bg->lbz = ilog2(opts->bz);
  if ((1 << bg->lbx) != opts->bx || (1 << bg->lby) != opts->by || (1 << bg->lbz) != opts->bz) return false;
  bg->nbx = (grid->nx + opts->bx - 1) / opts->bx;
  bg->nby = (grid->ny + opts->by - 1) / opts->by;
  bg->nbz = (grid->nz + opts->bz - 1) / opts->bz;
  bg->nbricks = (int64_t)bg->nbx * bg->nby * bg->nbz;
  // division constants: s = ceil(log2 d), m = floor(2^(32 + s) / d) - 2^32 + 1
  auto magic = [](uint32_t d, uint32_t &m, uint8_t &s) {
    int l = 0;
    while (((uint64_t)1 << l) < d) ++l;
    s = (uint8_t)l;
    m = (uint32_t)((((uint64_t)1 << (32 + l)) / d) - ((uint64_t)1 << 32) + 1);
  };
  magic((uint32_t)bg->nbx, bg->mbx, bg->sbx);
  magic((uint32_t)bg->nby, bg->mby, bg->sby);
  bg->ox = grid->origin[0];
  bg->oy = grid->origin[1];
  bg->oz = grid->origin[2];
  bg->hx = grid->spacing[0];
  bg->hy = grid->spacing[1];
  bg->hz = grid->spacing[2];
  bg->ihx = 1.f / grid->spacing[0];
  bg->ihy = 1.f / grid->spacing[1];
  bg->ihz = 1.f / grid->spacing[2];
  return true;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

WsLayout make_layout(int64_t n, int64_t nbricks, int64_t cap, bool partials) {
  WsLayout L;
  L.n = n;
  L.cap = cap;
  L.nbricks = nbricks;
  L.sort_blocks = (int)((cap + kSortTile - 1) / kSortTile);
  int bits = 0;
  while (bits < 32 && ((int64_t)1 << bits) < nbricks) ++bits;
  L.sort_passes = bits == 0 ? 1 : (bits + kRadixBits - 1) / kRadixBits;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  L.status = take(sizeof(DevStatus));
  L.evalrec = take(sizeof(EvalRec) * (size_t)n);
  L.cullrec = take(sizeof(CullRec) * (size_t)n);
  L.off = take(sizeof(uint32_t) * (size_t)(n + 1));
  L.runs = take(sizeof(uint32_t) * kRuns * (size_t)n);
  L.gbox = take(sizeof(uint32_t) * 4 * (size_t)n);
  L.key_brick = take(sizeof(uint32_t) * (size_t)cap);
  L.key_gid = take(sizeof(uint32_t) * (size_t)cap);
  L.keys_alt = take(sizeof(uint32_t) * (size_t)cap);
  L.vals_a = take(sizeof(uint32_t) * (size_t)cap);
  L.vals_b = take(sizeof(uint32_t) * (size_t)cap);
  L.list_gid = take(sizeof(uint32_t) * (size_t)cap);
  L.list_slot = take(sizeof(uint32_t) * (size_t)cap);
  L.brick_se = take(sizeof(uint32_t) * 2 * (size_t)nbricks);
  L.hist = take(sizeof(uint32_t) * (size_t)kRadix * (size_t)L.sort_blocks);
  // scan scratch: per-block key totals of the count scan, later the radix digit totals
  L.scan_tmp = take(std::max(sizeof(uint64_t) * (size_t)((n + kPrepThreads - 1) / kPrepThreads + 1),
                             sizeof(uint32_t) * (size_t)kRadix));
  L.partials = take(partials ? sizeof(float) * 12 * (size_t)cap : 0);
  L.total = o;
  return L;
}

// ---- argument checks -------------------------------------------------------------------------------

static int check_grid(const gs_grid_t *grid) {
  if (!grid) return fail(GS_ERR_INVALID_ARG, "grid is NULL");
  if (grid->nx <= 0 || grid->ny <= 0 || grid->nz <= 0)
    return fail(GS_ERR_INVALID_ARG, "grid dims must be positive (got %d x %d x %d)", grid->nx, grid->ny, grid->nz);
  if ((int64_t)grid->nx * grid->ny * grid->nz > ((int64_t)1 << 40))
    return fail(GS_ERR_INVALID_ARG, "grid too large");
  if (grid->nx > kMaxGridDim || grid->ny > kMaxGridDim || grid->nz > kMaxGridDim)
    return fail(GS_ERR_UNSUPPORTED, "grid dims above %d per axis are not supported", kMaxGridDim);
  for (int k = 0; k < 3; ++k) {
    if (!(grid->spacing[k] > 0.f) || !std::isfinite(grid->spacing[k]) || !std::isfinite(grid->origin[k]))
      return fail(GS_ERR_INVALID_ARG, "grid spacing must be positive and finite, origin finite");
  }
  return GS_OK;
}

static int check_opts(const gs_opts_t *opts) {
  if (!opts) return fail(GS_ERR_INVALID_ARG, "opts is NULL");
  if (opts->bx <= 0 || opts->by <= 0 || opts->bz <= 0) return fail(GS_ERR_INVALID_ARG, "brick dims must be positive");
  if (!brick_supported(opts->bx, opts->by, opts->bz))
    return fail(GS_ERR_UNSUPPORTED, "brick %dx%dx%d not supported by this library", opts->bx, opts->by, opts->bz);
  if (!(opts->cutoff > 0.f) || !std::isfinite(opts->cutoff)) return fail(GS_ERR_INVALID_ARG, "cutoff must be > 0");
  if (!(opts->eps > 0.f) || !std::isfinite(opts->eps)) return fail(GS_ERR_INVALID_ARG, "eps must be > 0 and finite");
  const uint32_t known = GS_FLAG_FORWARD_ONLY | GS_FLAG_BWD_ONE_BRICK | GS_FLAG_BWD_TWO_BRICKS |
                        GS_FLAG_BWD_WINDOW_256 | GS_FLAG_EMIT_STAGE_4K | GS_FLAG_EMIT_STAGE_6K;
  if ((opts->flags & ~known) != 0) return fail(GS_ERR_INVALID_ARG, "unknown flags");
  if ((opts->flags & GS_FLAG_EMIT_STAGE_4K) && (opts->flags & GS_FLAG_EMIT_STAGE_6K))
    return fail(GS_ERR_INVALID_ARG, "choose one emit stage flag");
  if ((opts->flags & GS_FLAG_BWD_ONE_BRICK) && (opts->flags & GS_FLAG_BWD_TWO_BRICKS))
    return fail(GS_ERR_INVALID_ARG, "choose one backward group flag");
  return GS_OK;
}

static int check_gaussians(const gs_gaussians_t *g) {
  if (!g) return fail(GS_ERR_INVALID_ARG, "gaussians is NULL");
  if (g->n < 0) return fail(GS_ERR_INVALID_ARG, "n must be >= 0");
  if (g->n >= ((int64_t)1 << 31)) return fail(GS_ERR_INVALID_ARG, "n must be < 2^31");
  if (g->n > 0 && (!g->mu || !g->log_scale || !g->quat || !g->amp))
    return fail(GS_ERR_INVALID_ARG, "mu, log_scale, quat and amp are required");
  return GS_OK;
}

// Scan table of a batch: Gaussians, bricks and volumes of the scans concatenated in order.  With
// zdown > 0 the observation offsets and the fit loss scales are filled in as well.
static int make_table(const gs_batch_t *bt, const gs_opts_t *opts, int32_t zdown, ScanTable *T) {
  int rc;
  if (!bt) return fail(GS_ERR_INVALID_ARG, "batch is NULL");
  if (bt->ns < 1 || bt->ns > GS_MAX_SCANS)
    return fail(GS_ERR_INVALID_ARG, "batch size must be in [1, %d] (got %d)", GS_MAX_SCANS, bt->ns);
  if (!bt->n || !bt->grid) return fail(GS_ERR_INVALID_ARG, "batch n and grid arrays are required");
  if ((rc = check_opts(opts))) return rc;
  std::memset(T, 0, sizeof *T);
  T->ns = bt->ns;
  T->bwd_bricks = bwd_bricks_of(opts->flags);
  int64_t g0 = 0, b0 = 0, p0 = 0, v0 = 0, o0 = 0;
  for (int k = 0; k < bt->ns; ++k) {
    const gs_grid_t *gr = &bt->grid[k];
    if ((rc = check_grid(gr))) return rc;
    if (bt->n[k] < 0) return fail(GS_ERR_INVALID_ARG, "scan %d: n must be >= 0", k);
    if (zdown > 0 && gr->nz % zdown != 0)
      return fail(GS_ERR_INVALID_ARG, "scan %d: nz (%d) must be a multiple of zdown (%d)", k, gr->nz, zdown);
    ScanDesc &sd = T->s[k];
    make_brick_grid(gr, opts, &sd.bg);
    sd.g0 = g0;
    sd.n = bt->n[k];
    sd.b0 = b0;
    sd.p0 = p0;
    sd.v0 = v0;
    sd.o0 = o0;
    const int64_t nvox = (int64_t)gr->nx * gr->ny * gr->nz;
    if (zdown > 0) {
      const int64_t nlr = nvox / zdown;
      sd.gscale = (float)(1.0 / ((double)zdown * (double)nlr));
      sd.lscale = (float)(1.0 / (double)nlr);
      o0 += nlr;
    }
    g0 += bt->n[k];
    b0 += sd.bg.nbricks;
    p0 += (sd.bg.nbricks + T->bwd_bricks - 1) / T->bwd_bricks;
    v0 += nvox;
  }
  T->n_total = g0;
  T->nbricks_total = b0;
  T->ngroups_total = p0;
  if (g0 >= ((int64_t)1 << 31)) return fail(GS_ERR_INVALID_ARG, "total Gaussian count must be < 2^31");
  if (b0 >= ((int64_t)1 << 31)) return fail(GS_ERR_INVALID_ARG, "too many bricks");
  if (v0 > ((int64_t)1 << 40)) return fail(GS_ERR_INVALID_ARG, "batch volumes too large");
  return GS_OK;
}

// Gaussian parameters of every scan: from the per-scan sets of the batch if it has them (then g must
// be NULL), else from the concatenated set g.
static int bind_gaussians(const gs_gaussians_t *g, const gs_batch_t *bt, ScanTable *T) {
  int rc;
  if (bt->sets) {
    if (g) return fail(GS_ERR_INVALID_ARG, "give either per-scan sets in the batch or one concatenated set, not both");
    for (int k = 0; k < T->ns; ++k) {
      const gs_gaussians_t &sk = bt->sets[k];
      if ((rc = check_gaussians(&sk))) return rc;
      if (sk.n != bt->n[k])
        return fail(GS_ERR_INVALID_ARG, "scan %d: set holds %lld Gaussians, batch n says %lld", k, (long long)sk.n,
                    (long long)bt->n[k]);
      ScanDesc &sd = T->s[k];
      sd.mu = sk.mu;
      sd.ls = sk.log_scale;
      sd.quat = sk.quat;
      sd.amp = sk.amp;
      sd.relax = sk.relax;
    }
    return GS_OK;
  }
  if ((rc = check_gaussians(g))) return rc;
  if (g->n != T->n_total)
    return fail(GS_ERR_INVALID_ARG, "the Gaussian set holds %lld Gaussians, the batch's scans %lld", (long long)g->n,
                (long long)T->n_total);
  for (int k = 0; k < T->ns; ++k) {
    ScanDesc &sd = T->s[k];
    const int64_t o = sd.g0;
    const bool any = g->n > 0;
    sd.mu = any ? g->mu + 3 * o : nullptr;
    sd.ls = any ? g->log_scale + 3 * o : nullptr;
    sd.quat = any ? g->quat + 4 * o : nullptr;
    sd.amp = any ? g->amp + o : nullptr;
    sd.relax = any && g->relax ? g->relax + o : nullptr;
  }
  return GS_OK;
}

static int check_common(const gs_gaussians_t *g, const gs_batch_t *bt, const gs_opts_t *opts, const gs_bins_t *bins,
                        int32_t zdown, ScanTable *T, WsLayout *L) {
  int rc;
  if ((rc = make_table(bt, opts, zdown, T)) || (rc = bind_gaussians(g, bt, T))) return rc;
  if (!bins || !bins->ws) return fail(GS_ERR_INVALID_ARG, "bins or bins->ws is NULL");
  if (bins->key_capacity < 0 || bins->key_capacity > (int64_t)0x7FFFFF00)
    return fail(GS_ERR_INVALID_ARG, "key_capacity must be in [0, 2^31 - 256]");
  *L = make_layout(T->n_total, T->nbricks_total, bins->key_capacity, !(opts->flags & GS_FLAG_FORWARD_ONLY));
  if (bins->ws_bytes < L->total)
    return fail(GS_ERR_INVALID_ARG, "workspace too small: %zu bytes given, %zu needed", bins->ws_bytes, L->total);
  return GS_OK;
}

// The one-scan batch of a single-scan call.
struct Single {
  int64_t n;
  gs_grid_t grid;
  gs_batch_t b;
  Single(int64_t n_, const gs_grid_t *g) : n(n_) {
    if (g) grid = *g;
    else std::memset(&grid, 0, sizeof grid);
    b.ns = 1;
    b.n = &n;
    b.grid = g ? &grid : nullptr;
    b.sets = nullptr;
  }
};

static int64_t bricks_at(const gs_grid_t &g, int bx) {
  return (int64_t)((g.nx + bx - 1) / bx) * ((g.ny + 7) / 8) * ((g.nz + 3) / 4);
}

// ---- static scratch for callers that cannot allocate ------------------------------------------------
//
// gs_render_fwd_noalloc keeps its binning workspace (forward-only layout) in this array.  Each GPU the
// library runs on holds its own copy until the process ends.  In host code `scratch` is only a
// stand-in for the symbol: its device address is looked up once per device, with that device
// current, and only that address is ever passed to kernels.  Nothing in the array has to start at
// zero: the binning writes every part of the workspace it later reads, the status block included.
static __device__ __align__(256) unsigned char scratch[GS_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_at[kMaxDevices];

static int static_scratch(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(GS_ERR_UNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_at[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(static scratch)");
    if (!p) return fail(GS_ERR_HIP, "hipGetSymbolAddress(static scratch) returned NULL");
    g_scratch_at[dev] = p;
  }
  *out = g_scratch_at[dev];
  return GS_OK;
}

// The largest key capacity whose forward-only layout fits the static scratch (-1: not even with 0).
static int64_t static_key_capacity(int64_t n, int64_t nbricks) {
  if (make_layout(n, nbricks, 0, false).total > GS_STATIC_SCRATCH_BYTES) return -1;
  int64_t lo = 0, hi = GS_STATIC_SCRATCH_BYTES / (4 * 7);
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo + 1) / 2;
    if (make_layout(n, nbricks, mid, false).total <= GS_STATIC_SCRATCH_BYTES) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ void k_copy_status(const DevStatus *src, gs_status_t *dst) {
  if (threadIdx.x == 0) {
    dst->n_keys = src->n_keys;
    dst->overflow = src->overflow;
    dst->nonfinite = src->nonfinite;
  }
}

}  // namespace gs

using namespace gs;

extern "C" {

const char *gs_last_error(void) { return g_last_error.c_str(); }

int gs_brick_supported(int32_t bx, int32_t by, int32_t bz) { return brick_supported(bx, by, bz) ? 1 : 0; }

int gs_workspace_size_batch(const gs_batch_t *batch, const gs_opts_t *opts, int64_t key_capacity, size_t *bytes) {
  if (!bytes) return fail(GS_ERR_INVALID_ARG, "bytes is NULL");
  if (key_capacity < 0) return fail(GS_ERR_INVALID_ARG, "key_capacity must be >= 0");
  ScanTable T;
  int rc = make_table(batch, opts, 0, &T);
  if (rc) return rc;
  *bytes = make_layout(T.n_total, T.nbricks_total, key_capacity, !(opts->flags & GS_FLAG_FORWARD_ONLY)).total;
  return GS_OK;
}

int gs_workspace_size(int64_t n, const gs_grid_t *grid, const gs_opts_t *opts, int64_t key_capacity, size_t *bytes) {
  if (n < 0) return fail(GS_ERR_INVALID_ARG, "n must be >= 0");
  Single one(n, grid);
  return gs_workspace_size_batch(&one.b, opts, key_capacity, bytes);
}

size_t gs_loss_scratch_bytes(int64_t nvox) { return sizeof(float) * (size_t)std::max(1, loss_blocks(nvox)); }

// step: the fit's per-scan step counters (advanced by the count scan), or NULL outside a fit step
// scan: run the count scan's second level (the emit does it for small sets when it follows)
static int bin_front(const gs_gaussians_t *g, const ScanTable &T, const gs_opts_t *opts, const gs_bins_t *bins,
                     const WsLayout &L, hipStream_t s, int32_t *step = nullptr, bool scan = true) {
  hipError_t e;
  if ((e = launch_prep_count(T, opts->cutoff, bins->ws, L, s)) != hipSuccess) return hip_fail(e, "prep_count");
  if (scan && (e = launch_scan_counts(bins->ws, L, step, T.ns, s)) != hipSuccess) return hip_fail(e, "scan_counts");
  return GS_OK;
}

int gs_bin_query_batch(const gs_gaussians_t *g, const gs_batch_t *batch, const gs_opts_t *opts, const gs_bins_t *bins,
                       void *stream, int64_t *n_keys) {
  ScanTable T;
  WsLayout L;
  int rc = check_common(g, batch, opts, bins, 0, &T, &L);
  if (rc) return rc;
  if (!n_keys) return fail(GS_ERR_INVALID_ARG, "n_keys is NULL");
  hipStream_t s = (hipStream_t)stream;
  if ((rc = bin_front(g, T, opts, bins, L, s))) return rc;
  DevStatus st;
  hipError_t e = hipMemcpyAsync(&st, (char *)bins->ws + L.status, sizeof st, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "gs_bin_query");
  *n_keys = st.n_keys;
  if (st.nonfinite) return fail(GS_ERR_NONFINITE, "non-finite parameter, zero quaternion or r <= 0");
  return GS_OK;
}

int gs_bin_query(const gs_gaussians_t *g, const gs_grid_t *grid, const gs_opts_t *opts, const gs_bins_t *bins,
                 void *stream, int64_t *n_keys) {
  Single one(g ? g->n : 0, grid);
  return gs_bin_query_batch(g, &one.b, opts, bins, stream, n_keys);
}

static int bin_all(const gs_gaussians_t *g, const ScanTable &T, const gs_opts_t *opts, const gs_bins_t *bins,
                   const WsLayout &L, hipStream_t s, int32_t *step = nullptr) {
  int rc;
  const bool fused = emit_scans(T.n_total);
  if ((rc = bin_front(g, T, opts, bins, L, s, step, !fused))) return rc;
  hipError_t e;
  if ((e = launch_emit(T, opts->cutoff, opts->flags, bins->ws, L, fused ? step : nullptr, s)) != hipSuccess)
    return hip_fail(e, "emit");
  if ((e = launch_sort(T, bins->ws, L, s)) != hipSuccess) return hip_fail(e, "sort");
  return GS_OK;
}

int gs_bin_batch(const gs_gaussians_t *g, const gs_batch_t *batch, const gs_opts_t *opts, const gs_bins_t *bins,
                 void *stream) {
  ScanTable T;
  WsLayout L;
  int rc = check_common(g, batch, opts, bins, 0, &T, &L);
  if (rc) return rc;
  return bin_all(g, T, opts, bins, L, (hipStream_t)stream);
}

int gs_bin(const gs_gaussians_t *g, const gs_grid_t *grid, const gs_opts_t *opts, const gs_bins_t *bins,
           void *stream) {
  Single one(g ? g->n : 0, grid);
  return gs_bin_batch(g, &one.b, opts, bins, stream);
}

int gs_render_fwd_batch(const gs_gaussians_t *g, const gs_batch_t *batch, const gs_opts_t *opts, const gs_bins_t *bins,
                        float *I, float *W, void *stream) {
  ScanTable T;
  WsLayout L;
  int rc = check_common(g, batch, opts, bins, 0, &T, &L);
  if (rc) return rc;
  if (!I) return fail(GS_ERR_INVALID_ARG, "I is NULL");
  hipError_t e = launch_fwd(T, opts->bx, opts->cutoff, opts->eps, bins->ws, L, I, W, (hipStream_t)stream);
  return e == hipSuccess ? GS_OK : hip_fail(e, "render_fwd");
}

int gs_render_fwd(const gs_gaussians_t *g, const gs_grid_t *grid, const gs_opts_t *opts, const gs_bins_t *bins,
                  float *I, float *W, void *stream) {
  Single one(g ? g->n : 0, grid);
  return gs_render_fwd_batch(g, &one.b, opts, bins, I, W, stream);
}

int gs_count_pairs_batch(const gs_gaussians_t *g, const gs_batch_t *batch, const gs_opts_t *opts,
                         const gs_bins_t *bins, int64_t *d_count, void *stream) {
  ScanTable T;
  WsLayout L;
  int rc = check_common(g, batch, opts, bins, 0, &T, &L);
  if (rc) return rc;
  if (!d_count) return fail(GS_ERR_INVALID_ARG, "d_count is NULL");
  hipError_t e = launch_count_pairs(T, opts->bx, opts->cutoff, bins->ws, L, d_count, (hipStream_t)stream);
  return e == hipSuccess ? GS_OK : hip_fail(e, "count_pairs");
}

int gs_count_pairs(const gs_gaussians_t *g, const gs_grid_t *grid, const gs_opts_t *opts, const gs_bins_t *bins,
                   int64_t *d_count, void *stream) {
  Single one(g ? g->n : 0, grid);
  return gs_count_pairs_batch(g, &one.b, opts, bins, d_count, stream);
}

int gs_count_evals(const gs_gaussians_t *g, const gs_grid_t *grid, const gs_opts_t *opts, const gs_bins_t *bins,
                   int64_t *d_counts, void *stream) {
  Single one(g ? g->n : 0, grid);
  ScanTable T;
  WsLayout L;
  int rc = check_common(g, &one.b, opts, bins, 0, &T, &L);
  if (rc) return rc;
  if (!d_counts) return fail(GS_ERR_INVALID_ARG, "d_counts is NULL");
  hipError_t e = launch_count_evals(T, opts->bx, opts->flags, opts->cutoff, bins->ws, L, d_counts, (hipStream_t)stream);
  return e == hipSuccess ? GS_OK : hip_fail(e, "count_evals");
}

int gs_render_bwd_batch(const gs_gaussians_t *g, const gs_batch_t *batch, const gs_opts_t *opts, const gs_bins_t *bins,
                        const float *I, const float *W, const float *dL_dI, const gs_grads_t *grads, void *stream) {
  ScanTable T;
  WsLayout L;
  int rc = check_common(g, batch, opts, bins, 0, &T, &L);
  if (rc) return rc;
  if (batch->sets) return fail(GS_ERR_INVALID_ARG, "the backward takes one concatenated Gaussian set");
  if (opts->flags & GS_FLAG_FORWARD_ONLY) return fail(GS_ERR_INVALID_ARG, "forward-only workspace: no backward");
  if (!I || !W || !dL_dI || !grads) return fail(GS_ERR_INVALID_ARG, "I, W, dL_dI and grads are required");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_bwd(T, opts->bx, opts->flags, opts->cutoff, opts->eps, bins->ws, L, I, W, dL_dI, s);
  if (e != hipSuccess) return hip_fail(e, "render_bwd");
  e = launch_reduce_chain(*g, bins->ws, L, *grads, s);
  return e == hipSuccess ? GS_OK : hip_fail(e, "reduce_chain");
}

int gs_render_bwd(const gs_gaussians_t *g, const gs_grid_t *grid, const gs_opts_t *opts, const gs_bins_t *bins,
                  const float *I, const float *W, const float *dL_dI, const gs_grads_t *grads, void *stream) {
  Single one(g ? g->n : 0, grid);
  return gs_render_bwd_batch(g, &one.b, opts, bins, I, W, dL_dI, grads, stream);
}

int gs_loss_mse(const float *I, const float *T, int64_t nvox, float *dL_dI, float *loss, void *scratch,
                size_t scratch_bytes, void *stream) {
  if (nvox <= 0 || !I || !T || !dL_dI || !loss || !scratch)
    return fail(GS_ERR_INVALID_ARG, "gs_loss_mse: null pointer or nvox <= 0");
  if (scratch_bytes < gs_loss_scratch_bytes(nvox)) return fail(GS_ERR_INVALID_ARG, "gs_loss_mse: scratch too small");
  hipError_t e = launch_loss_mse(I, T, nvox, dL_dI, loss, scratch, (hipStream_t)stream);
  return e == hipSuccess ? GS_OK : hip_fail(e, "loss_mse");
}

int gs_loss_l1_zmean(const float *I, const float *obs, const gs_grid_t *hr, int32_t zdown, float *dL_dI, float *loss,
                     void *scratch, size_t scratch_bytes, void *stream) {
  int rc = check_grid(hr);
  if (rc) return rc;
  if (zdown <= 0 || hr->nz % zdown != 0) return fail(GS_ERR_INVALID_ARG, "nz must be a positive multiple of zdown");
  if (!I || !obs || !dL_dI || !loss || !scratch) return fail(GS_ERR_INVALID_ARG, "gs_loss_l1_zmean: null pointer");
  int64_t nlr = (int64_t)hr->nx * hr->ny * (hr->nz / zdown);
  if (scratch_bytes < gs_loss_scratch_bytes(nlr)) return fail(GS_ERR_INVALID_ARG, "gs_loss_l1_zmean: scratch too small");
  hipError_t e = launch_loss_l1z(I, obs, hr->nx, hr->ny, hr->nz, zdown, dL_dI, loss, scratch, (hipStream_t)stream);
  return e == hipSuccess ? GS_OK : hip_fail(e, "loss_l1z");
}

static int check_state(const gs_fit_state_t *st, const gs_grads_t *gr) {
  if (!st || !gr) return fail(GS_ERR_INVALID_ARG, "state or grads is NULL");
  if (st->n < 0) return fail(GS_ERR_INVALID_ARG, "n must be >= 0");
  if (st->n > 0 && (!st->mu || !st->log_scale || !st->quat || !st->amp || !st->m || !st->v))
    return fail(GS_ERR_INVALID_ARG, "state arrays mu, log_scale, quat, amp, m, v are required");
  if (!st->step) return fail(GS_ERR_INVALID_ARG, "step is required");
  if (st->n > 0 && (!gr->d_mu || !gr->d_log_scale || !gr->d_quat || !gr->d_amp))
    return fail(GS_ERR_INVALID_ARG, "gradients d_mu, d_log_scale, d_quat, d_amp are required");
  if (st->n > 0 && st->relax && !gr->d_relax) return fail(GS_ERR_INVALID_ARG, "d_relax is required when relax is set");
  return GS_OK;
}

int gs_adam_step(const gs_fit_state_t *st, const gs_grads_t *grads, const gs_adam_t *hp, const gs_bins_t *bins,
                 void *stream) {
  int rc = check_state(st, grads);
  if (rc) return rc;
  if (!hp) return fail(GS_ERR_INVALID_ARG, "hp is NULL");
  const void *status = bins && bins->ws ? bins->ws : nullptr;  // status block is at offset 0
  hipError_t e = launch_adam(*st, *grads, *hp, status, (hipStream_t)stream);
  return e == hipSuccess ? GS_OK : hip_fail(e, "adam");
}

size_t gs_fit_scratch_bytes_batch(const gs_batch_t *batch) {
  if (!batch || batch->ns < 1 || batch->ns > GS_MAX_SCANS || !batch->grid) return 0;
  // fused path: one float per brick of every scan at the narrowest supported brick (the most bricks);
  // separate loss path: the loss reduction of the largest scan
  int64_t bricks = 0, blocks = 1;
  for (int k = 0; k < batch->ns; ++k) {
    const gs_grid_t &g = batch->grid[k];
    if (g.nx <= 0 || g.ny <= 0 || g.nz <= 0) return 0;
    bricks += bricks_at(g, 4);
    blocks = std::max<int64_t>(blocks, loss_blocks((int64_t)g.nx * g.ny * g.nz));
  }
  return sizeof(float) * (size_t)std::max(bricks, blocks);
}

size_t gs_fit_scratch_bytes(const gs_grid_t *hr) {
  if (!hr) return 0;
  Single one(0, hr);
  return gs_fit_scratch_bytes_batch(&one.b);
}

int gs_fit_step_batch(const gs_fit_state_t *st, const float *lr_obs, const gs_batch_t *batch, const gs_fit_opts_t *fo,
                      const gs_bins_t *bins, const gs_fit_buffers_t *buf, void *stream) {
  if (!fo || !buf || !lr_obs) return fail(GS_ERR_INVALID_ARG, "fit opts, buffers and lr_obs are required");
  int rc = check_state(st, &buf->grads);
  if (rc) return rc;
  if (fo->loss != 0) return fail(GS_ERR_UNSUPPORTED, "only loss 0 (L1 on the z-mean) is supported");
  if (fo->zdown <= 0) return fail(GS_ERR_INVALID_ARG, "zdown must be positive");
  if (batch && batch->sets) return fail(GS_ERR_INVALID_ARG, "the fit takes one concatenated Gaussian set");
  if (fo->opts.flags & GS_FLAG_FORWARD_ONLY) return fail(GS_ERR_INVALID_ARG, "forward-only workspace: no fit");
  gs_gaussians_t g{st->n, st->mu, st->log_scale, st->quat, st->amp, st->relax};
  ScanTable T;
  WsLayout L;
  if ((rc = check_common(&g, batch, &fo->opts, bins, fo->zdown, &T, &L))) return rc;
  if (!buf->I || !buf->W || !buf->loss || !buf->scratch) return fail(GS_ERR_INVALID_ARG, "fit buffers incomplete");
  const size_t need = gs_fit_scratch_bytes_batch(batch);
  if (buf->scratch_bytes < need)
    return fail(GS_ERR_INVALID_ARG, "fit scratch too small: %zu bytes given, %zu needed", buf->scratch_bytes, need);
  const bool fused = fo->zdown == fo->opts.bz;
  if (!fused && !buf->dL_dI)
    return fail(GS_ERR_INVALID_ARG, "dL_dI is required when zdown differs from the brick depth");
  hipStream_t s = (hipStream_t)stream;
  if ((rc = bin_all(&g, T, &fo->opts, bins, L, s, st->step))) return rc;
  const gs_opts_t &o = fo->opts;
  hipError_t e = launch_fwd(T, o.bx, o.cutoff, o.eps, bins->ws, L, buf->I, buf->W, s);
  if (e != hipSuccess) return hip_fail(e, "render_fwd");
  if (fused) {
    // the z-mean groups coincide with the brick's z extent: loss fused into the backward's staging,
    // gradient reduction fused with Adam
    float *loss_part = (float *)buf->scratch;
    e = launch_bwd_fit(T, o.bx, o.flags, o.cutoff, o.eps, bins->ws, L, buf->I, buf->W, lr_obs, loss_part, s);
    if (e != hipSuccess) return hip_fail(e, "render_bwd");
    e = launch_reduce_adam(T, *st, bins->ws, L, buf->grads, fo->adam, loss_part, buf->loss, s);
    return e == hipSuccess ? GS_OK : hip_fail(e, "reduce_adam");
  }
  for (int k = 0; k < T.ns; ++k) {
    const ScanDesc &sd = T.s[k];
    e = launch_loss_l1z(buf->I + sd.v0, lr_obs + sd.o0, sd.bg.nx, sd.bg.ny, sd.bg.nz, fo->zdown, buf->dL_dI + sd.v0,
                        buf->loss + k, buf->scratch, s, (const DevStatus *)((char *)bins->ws + L.status));
    if (e != hipSuccess) return hip_fail(e, "loss_l1z");
  }
  e = launch_bwd(T, o.bx, o.flags, o.cutoff, o.eps, bins->ws, L, buf->I, buf->W, buf->dL_dI, s);
  if (e != hipSuccess) return hip_fail(e, "render_bwd");
  e = launch_reduce_adam(T, *st, bins->ws, L, buf->grads, fo->adam, nullptr, buf->loss, s);
  return e == hipSuccess ? GS_OK : hip_fail(e, "reduce_adam");
}

int gs_fit_step(const gs_fit_state_t *st, const float *lr_obs, const gs_fit_opts_t *fo, const gs_bins_t *bins,
                const gs_fit_buffers_t *buf, void *stream) {
  if (!fo) return fail(GS_ERR_INVALID_ARG, "fit opts are required");
  Single one(st ? st->n : 0, &fo->hr);
  return gs_fit_step_batch(st, lr_obs, &one.b, fo, bins, buf, stream);
}

int gs_render_fwd_noalloc(const gs_gaussians_t *g, const gs_grid_t *grid, const gs_opts_t *opts, float *I, float *W,
                          gs_status_t *d_status, void *stream) {
  Single one(g ? g->n : 0, grid);
  ScanTable T;
  int rc;
  if ((rc = make_table(&one.b, opts, 0, &T)) || (rc = bind_gaussians(g, &one.b, &T))) return rc;
  if (!I) return fail(GS_ERR_INVALID_ARG, "I is NULL");
  const int64_t cap = static_key_capacity(T.n_total, T.nbricks_total);
  if (cap < 0)
    return fail(GS_ERR_INVALID_ARG,
                "%lld Gaussians on %lld bricks need %zu bytes of workspace before any key; the static scratch "
                "holds %llu bytes",
                (long long)T.n_total, (long long)T.nbricks_total, make_layout(T.n_total, T.nbricks_total, 0, false).total,
                (unsigned long long)GS_STATIC_SCRATCH_BYTES);
  void *ws = nullptr;
  if ((rc = static_scratch(&ws))) return rc;
  gs_opts_t o = *opts;
  o.flags |= GS_FLAG_FORWARD_ONLY;
  const gs_bins_t bins{ws, (size_t)GS_STATIC_SCRATCH_BYTES, cap};
  const WsLayout L = make_layout(T.n_total, T.nbricks_total, cap, false);
  hipStream_t s = (hipStream_t)stream;
  if ((rc = bin_all(g, T, &o, &bins, L, s))) return rc;
  hipError_t e = launch_fwd(T, o.bx, o.cutoff, o.eps, ws, L, I, W, s);
  if (e != hipSuccess) return hip_fail(e, "render_fwd");
  if (d_status) {
    k_copy_status<<<1, 64, 0, s>>>((const DevStatus *)((char *)ws + L.status), d_status);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "copy_status");
  }
  return GS_OK;
}

int gs_status(const gs_bins_t *bins, void *stream, gs_status_t *out) {
  if (!bins || !bins->ws || !out) return fail(GS_ERR_INVALID_ARG, "bins, bins->ws and out are required");
  DevStatus st;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(&st, bins->ws, sizeof st, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "gs_status");
  out->n_keys = st.n_keys;
  out->overflow = st.overflow;
  out->nonfinite = st.nonfinite;
  if (st.overflow)
    return fail(GS_ERR_CAPACITY, "%lld keys exceed the key capacity %lld", (long long)st.n_keys,
                (long long)bins->key_capacity);
  if (st.nonfinite) return fail(GS_ERR_NONFINITE, "non-finite parameter, zero quaternion or r <= 0");
  return GS_OK;
}

int gs_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = on != 0;
  return GS_OK;
}

int gs_profile_reset(void) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto &r : g_prof_pending) {
    g_prof_pool.push_back(r.a);
    g_prof_pool.push_back(r.b);
  }
  g_prof_pending.clear();
  g_prof_acc.clear();
  return GS_OK;
}

int gs_profile_read(void *stream, int cap, char (*names)[48], int64_t *launches, double *total_ms, int *n_out) {
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "gs_profile_read");
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto &r : g_prof_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      bool found = false;
      for (auto &a : g_prof_acc)
        if (a.first == r.name) {
          a.second.first += 1;
          a.second.second += ms;
          found = true;
        }
      if (!found) g_prof_acc.push_back({r.name, {1, (double)ms}});
    }
    g_prof_pool.push_back(r.a);
    g_prof_pool.push_back(r.b);
  }
  g_prof_pending.clear();
  int k = 0;
  for (auto &a : g_prof_acc) {
    if (k >= cap) break;
    if (names) {
      std::strncpy(names[k], a.first.c_str(), 47);
      names[k][47] = 0;
    }
    if (launches) launches[k] = a.second.first;
    if (total_ms) total_ms[k] = a.second.second;
    ++k;
  }
  if (n_out) *n_out = k;
  return GS_OK;
}

}  // extern "C"
