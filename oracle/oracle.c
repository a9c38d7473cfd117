/*
 * Oracle: plain CPU definition of the order-independent Gaussian-to-voxel renderer and of its
 * gradient, in FP64 (or long double when built with -DOG_LONG_DOUBLE).
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load this library. It shares no code, header, table or helper with the GPU library,
 * and nothing of the GPU library is called from here.
 *
 * What it computes, following the paper:
 *   - Parameters (§3.1, "MRI-Tailored Gaussian Parameters"): per Gaussian a position mu (3), a
 *     covariance given by 3 log-scales s and a quaternion q (the "covariance:7" of the parameter
 *     count), an amplitude A and a relaxation factor r.  Sigma = R(q) diag(exp(2 s)) R(q)^T with
 *     R(q) the rotation of the normalised quaternion (w, x, y, z).
 *   - Spatial weight (§3.2, equation after Eq. (rendering)):
 *       w_i(p) = r_i exp(-1/2 (p - mu_i)^T Sigma_i^{-1} (p - mu_i)),
 *     truncated to the 3-sigma Mahalanobis ellipsoid used by the rasterizer (§3.3): the pair
 *     (p, i) contributes only if d^2 = (p - mu_i)^T Sigma_i^{-1} (p - mu_i) <= cutoff^2, cutoff = 3.
 *   - Normalised aggregation (§3.2, Eq. (rendering)) with a small eps in the denominator:
 *       W(p) = sum_i w_i(p),  S(p) = sum_i A_i w_i(p),  I(p) = S(p) / (W(p) + eps).
 *   - Gradients (§3.3, the two gradient equations), with W replaced by W + eps:
 *       dL/dA_i     = sum_p dL/dI(p) w_i(p) / (W(p) + eps)
 *       dL/dtheta_i = sum_p dL/dI(p) (A_i - I(p)) / (W(p) + eps) dw_i(p)/dtheta_i,
 *     summed over every voxel in the support of Gaussian i, with
 *       dw/dmu = w P delta,  dw/dP = -1/2 w delta delta^T,  dw/dr = exp(-d^2/2),
 *     P = Sigma^{-1}, delta = p - mu, and then the chain rule from P to (s, q).
 *
 * The loops are the plain definition: for every Gaussian, visit every voxel of its axis-aligned
 * index box (the 3-sigma box padded by one voxel), evaluate d^2 and apply the per-pair predicate.
 * No bricks, no sorting, no blocking.  OpenMP splits the forward over z-slabs (each thread owns its
 * output slices and visits the Gaussians in index order, so every voxel sums in ascending Gaussian
 * order) and the backward over Gaussians (read-only inputs); both are deterministic.
 *
 * Grid convention: voxel (ix, iy, iz) has centre origin + spacing * (ix, iy, iz); volumes are
 * stored [nz][ny][nx] with x fastest.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#ifdef OG_LONG_DOUBLE
typedef long double real_t;
#define R_EXP expl
#define R_SQRT sqrtl
#define R_CEIL ceill
#define R_FLOOR floorl
#define R_FABS fabsl
#else
typedef double real_t;
#define R_EXP exp
#define R_SQRT sqrt
#define R_CEIL ceil
#define R_FLOOR floor
#define R_FABS fabs
#endif

typedef struct {
  real_t mu[3];
  real_t qhat[4];   /* normalised quaternion (w, x, y, z) */
  real_t qnorm;     /* norm of the raw quaternion */
  real_t R[3][3];   /* rotation of qhat */
  real_t ev[3];     /* exp(2 s_k): variance along principal axis k */
  real_t Sig[3][3]; /* covariance R diag(ev) R^T */
  real_t P[3][3];   /* precision R diag(1/ev) R^T */
  real_t A, r;
  int lo[3], hi[3]; /* inclusive voxel index box; empty when lo > hi on some axis */
} og_gauss_t;

typedef struct {
  int n[3];
  real_t o[3], h[3];
} og_grid_t;

/* Rotation matrix of a unit quaternion (w, x, y, z). */
static void rotation_of(const real_t q[4], real_t R[3][3]) {
  real_t w = q[0], x = q[1], y = q[2], z = q[3];
  R[0][0] = 1 - 2 * (y * y + z * z);
  R[0][1] = 2 * (x * y - w * z);
  R[0][2] = 2 * (x * z + w * y);
  R[1][0] = 2 * (x * y + w * z);
  R[1][1] = 1 - 2 * (x * x + z * z);
  R[1][2] = 2 * (y * z - w * x);
  R[2][0] = 2 * (x * z - w * y);
  R[2][1] = 2 * (y * z + w * x);
  R[2][2] = 1 - 2 * (x * x + y * y);
}

/* One axis of the index box: the voxels whose centres lie within [m - a, m + a], padded by one
 * voxel on each side so that rounding never drops a voxel; the per-pair predicate decides. */
static void index_range(real_t m, real_t a, real_t o, real_t h, int n, int *lo, int *hi) {
  real_t l = R_CEIL((m - a - o) / h) - 1;
  real_t u = R_FLOOR((m + a - o) / h) + 1;
  if (l < 0) l = 0;
  if (u > (real_t)(n - 1)) u = (real_t)(n - 1);
  if (!(l <= u)) { /* empty (also catches NaN) */
    *lo = 1;
    *hi = 0;
    return;
  }
  *lo = (int)l;
  *hi = (int)u;
}

/* Build the per-Gaussian quantities.  Returns 0, or -1 for a non-finite input or a zero
 * quaternion. */
static int setup_gauss(og_gauss_t *G, int64_t i, const float *mu, const float *log_scale, const float *quat,
                       const float *amp, const float *relax, const og_grid_t *g, real_t cutoff) {
  real_t q[4], nrm2 = 0;
  for (int k = 0; k < 4; ++k) {
    q[k] = (real_t)quat[4 * i + k];
    nrm2 += q[k] * q[k];
  }
  for (int k = 0; k < 3; ++k) {
    G->mu[k] = (real_t)mu[3 * i + k];
    if (!isfinite((double)G->mu[k]) || !isfinite((double)log_scale[3 * i + k])) return -1;
  }
  if (!(nrm2 > 0) || !isfinite((double)nrm2)) return -1;
  G->qnorm = R_SQRT(nrm2);
  for (int k = 0; k < 4; ++k) G->qhat[k] = q[k] / G->qnorm;
  rotation_of(G->qhat, G->R);
  for (int k = 0; k < 3; ++k) G->ev[k] = R_EXP(2 * (real_t)log_scale[3 * i + k]);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      real_t s = 0, p = 0;
      for (int k = 0; k < 3; ++k) {
        s += G->R[a][k] * G->ev[k] * G->R[b][k];
        p += G->R[a][k] / G->ev[k] * G->R[b][k];
      }
      G->Sig[a][b] = s;
      G->P[a][b] = p;
    }
  G->A = (real_t)amp[i];
  G->r = relax ? (real_t)relax[i] : 1;
  if (!isfinite((double)G->A) || !isfinite((double)G->r)) return -1;
  for (int k = 0; k < 3; ++k) {
    real_t a = cutoff * R_SQRT(G->Sig[k][k]);
    index_range(G->mu[k], a, g->o[k], g->h[k], g->n[k], &G->lo[k], &G->hi[k]);
  }
  return 0;
}

static int setup_all(og_gauss_t *G, int64_t n, const float *mu, const float *log_scale, const float *quat,
                     const float *amp, const float *relax, const og_grid_t *g, real_t cutoff, int nthreads) {
  int bad = 0;
#pragma omp parallel for num_threads(nthreads) schedule(static) reduction(| : bad)
  for (int64_t i = 0; i < n; ++i) bad |= (setup_gauss(&G[i], i, mu, log_scale, quat, amp, relax, g, cutoff) != 0);
  return bad ? -1 : 0;
}

static void make_grid(og_grid_t *g, int nx, int ny, int nz, const double *origin, const double *spacing) {
  g->n[0] = nx;
  g->n[1] = ny;
  g->n[2] = nz;
  for (int k = 0; k < 3; ++k) {
    g->o[k] = (real_t)origin[k];
    g->h[k] = (real_t)spacing[k];
  }
}

/* Squared Mahalanobis distance of voxel (ix, iy, iz) from Gaussian G; also returns delta. */
static real_t maha2(const og_gauss_t *G, const og_grid_t *g, int ix, int iy, int iz, real_t d[3]) {
  d[0] = g->o[0] + g->h[0] * ix - G->mu[0];
  d[1] = g->o[1] + g->h[1] * iy - G->mu[1];
  d[2] = g->o[2] + g->h[2] * iz - G->mu[2];
  real_t s = 0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) s += d[a] * G->P[a][b] * d[b];
  return s;
}

static int64_t vidx(const og_grid_t *g, int ix, int iy, int iz) {
  return ((int64_t)iz * g->n[1] + iy) * g->n[0] + ix;
}

/* ---------------------------------------------------------------------------------------------
 * Per-Gaussian geometry, exported for the pins: R, Sigma and P (row-major 3x3 each).
 */
int og_frames(int64_t n, const float *log_scale, const float *quat, double *R, double *Sig, double *P) {
  float zero3[3] = {0, 0, 0}, one = 1;
  og_grid_t g;
  double o[3] = {0, 0, 0}, h[3] = {1, 1, 1};
  make_grid(&g, 1, 1, 1, o, h);
  for (int64_t i = 0; i < n; ++i) {
    og_gauss_t G;
    /* position, amplitude and relaxation do not enter the frame */
    if (setup_gauss(&G, 0, zero3, log_scale + 3 * i, quat + 4 * i, &one, NULL, &g, 3) != 0) return -1;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        R[9 * i + 3 * a + b] = (double)G.R[a][b];
        Sig[9 * i + 3 * a + b] = (double)G.Sig[a][b];
        P[9 * i + 3 * a + b] = (double)G.P[a][b];
      }
  }
  return 0;
}

/* ---------------------------------------------------------------------------------------------
 * Forward render on the whole grid (§3.2 Eq. (rendering), truncated per §3.3).
 * I, W, S: [nz][ny][nx] outputs; any of W, S may be NULL.  cutoff may be +inf (no truncation).
 */
int og_render(int64_t n, const float *mu, const float *log_scale, const float *quat, const float *amp,
              const float *relax, int nx, int ny, int nz, const double *origin, const double *spacing, double cutoff,
              double eps, double *I, double *W, double *S, int nthreads) {
  og_grid_t g;
  make_grid(&g, nx, ny, nz, origin, spacing);
  int64_t V = (int64_t)nx * ny * nz;
  og_gauss_t *G = (og_gauss_t *)malloc(sizeof(og_gauss_t) * (size_t)(n > 0 ? n : 1));
  real_t *Wacc = (real_t *)calloc((size_t)V, sizeof(real_t));
  real_t *Sacc = (real_t *)calloc((size_t)V, sizeof(real_t));
  if (!G || !Wacc || !Sacc) {
    free(G);
    free(Wacc);
    free(Sacc);
    return -2;
  }
  int rc = setup_all(G, n, mu, log_scale, quat, amp, relax, &g, (real_t)cutoff, nthreads);
  real_t c2 = (real_t)cutoff * (real_t)cutoff;
  if (rc == 0) {
#pragma omp parallel num_threads(nthreads)
    {
      int T = omp_get_num_threads(), t = omp_get_thread_num();
      int z0 = (int)((int64_t)nz * t / T), z1 = (int)((int64_t)nz * (t + 1) / T); /* owned slab [z0, z1) */
      for (int64_t i = 0; i < n; ++i) {
        const og_gauss_t *Gi = &G[i];
        if (Gi->lo[0] > Gi->hi[0] || Gi->lo[1] > Gi->hi[1] || Gi->lo[2] > Gi->hi[2]) continue;
        int za = Gi->lo[2] > z0 ? Gi->lo[2] : z0;
        int zb = Gi->hi[2] < z1 - 1 ? Gi->hi[2] : z1 - 1;
        for (int iz = za; iz <= zb; ++iz)
          for (int iy = Gi->lo[1]; iy <= Gi->hi[1]; ++iy)
            for (int ix = Gi->lo[0]; ix <= Gi->hi[0]; ++ix) {
              real_t d[3];
              real_t d2 = maha2(Gi, &g, ix, iy, iz, d);
              if (d2 <= c2) {
                real_t w = Gi->r * R_EXP(-d2 / 2);
                int64_t v = vidx(&g, ix, iy, iz);
                Wacc[v] += w;
                Sacc[v] += Gi->A * w;
              }
            }
      }
    }
    for (int64_t v = 0; v < V; ++v) {
      I[v] = (double)(Sacc[v] / (Wacc[v] + (real_t)eps));
      if (W) W[v] = (double)Wacc[v];
      if (S) S[v] = (double)Sacc[v];
    }
  }
  free(G);
  free(Wacc);
  free(Sacc);
  return rc;
}

/* Forward at a list of voxels (flat indices into [nz][ny][nx]): every Gaussian whose index box
 * holds the voxel is tested with the same predicate, in ascending Gaussian order. */
int og_render_points(int64_t n, const float *mu, const float *log_scale, const float *quat, const float *amp,
                     const float *relax, int nx, int ny, int nz, const double *origin, const double *spacing,
                     double cutoff, double eps, int64_t npts, const int64_t *vox, double *I, double *W, double *S,
                     int nthreads) {
  og_grid_t g;
  make_grid(&g, nx, ny, nz, origin, spacing);
  og_gauss_t *G = (og_gauss_t *)malloc(sizeof(og_gauss_t) * (size_t)(n > 0 ? n : 1));
  if (!G) return -2;
  int rc = setup_all(G, n, mu, log_scale, quat, amp, relax, &g, (real_t)cutoff, nthreads);
  real_t c2 = (real_t)cutoff * (real_t)cutoff;
  if (rc == 0) {
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 4)
    for (int64_t k = 0; k < npts; ++k) {
      int64_t v = vox[k];
      int ix = (int)(v % nx), iy = (int)((v / nx) % ny), iz = (int)(v / ((int64_t)nx * ny));
      real_t Wv = 0, Sv = 0;
      for (int64_t i = 0; i < n; ++i) {
        const og_gauss_t *Gi = &G[i];
        if (ix < Gi->lo[0] || ix > Gi->hi[0] || iy < Gi->lo[1] || iy > Gi->hi[1] || iz < Gi->lo[2] ||
            iz > Gi->hi[2])
          continue;
        real_t d[3];
        real_t d2 = maha2(Gi, &g, ix, iy, iz, d);
        if (d2 <= c2) {
          real_t w = Gi->r * R_EXP(-d2 / 2);
          Wv += w;
          Sv += Gi->A * w;
        }
      }
      I[k] = (double)(Sv / (Wv + (real_t)eps));
      if (W) W[k] = (double)Wv;
      if (S) S[k] = (double)Sv;
    }
  }
  free(G);
  return rc;
}

/* ---------------------------------------------------------------------------------------------
 * Chain rule from the precision matrix P = R diag(exp(-2 s)) R^T to (s, q).
 * Gp is dL/dP for a symmetric P (entries treated as independent, Gp symmetric).
 *   dL/dD  = diag(R^T Gp R),  D_k = exp(-2 s_k)  ->  dL/ds_k = -2 D_k (R^T Gp R)_kk
 *   dL/dR  = 2 Gp R D
 *   dL/dqhat from dR through the quaternion-to-rotation formula, then through qhat = q / |q|.
 */
static void chain_to_scale_quat(const og_gauss_t *G, const real_t Gp[3][3], real_t ds[3], real_t dq[4]) {
  real_t D[3], RtGR[3];
  for (int k = 0; k < 3; ++k) D[k] = 1 / G->ev[k];
  for (int k = 0; k < 3; ++k) {
    real_t s = 0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) s += G->R[a][k] * Gp[a][b] * G->R[b][k];
    RtGR[k] = s;
    ds[k] = -2 * D[k] * RtGR[k];
  }
  real_t dR[3][3];
  for (int a = 0; a < 3; ++a)
    for (int k = 0; k < 3; ++k) {
      real_t s = 0;
      for (int b = 0; b < 3; ++b) s += Gp[a][b] * G->R[b][k];
      dR[a][k] = 2 * s * D[k];
    }
  real_t w = G->qhat[0], x = G->qhat[1], y = G->qhat[2], z = G->qhat[3];
  real_t gw = 2 * (-z * dR[0][1] + y * dR[0][2] + z * dR[1][0] - x * dR[1][2] - y * dR[2][0] + x * dR[2][1]);
  real_t gx = 2 * (y * dR[0][1] + z * dR[0][2] + y * dR[1][0] - 2 * x * dR[1][1] - w * dR[1][2] + z * dR[2][0] +
                   w * dR[2][1] - 2 * x * dR[2][2]);
  real_t gy = 2 * (-2 * y * dR[0][0] + x * dR[0][1] + w * dR[0][2] + x * dR[1][0] + z * dR[1][2] - w * dR[2][0] +
                   z * dR[2][1] - 2 * y * dR[2][2]);
  real_t gz = 2 * (-2 * z * dR[0][0] - w * dR[0][1] + x * dR[0][2] + w * dR[1][0] - 2 * z * dR[1][1] +
                   y * dR[1][2] + x * dR[2][0] + y * dR[2][1]);
  real_t gq[4] = {gw, gx, gy, gz};
  real_t dot = 0;
  for (int k = 0; k < 4; ++k) dot += G->qhat[k] * gq[k];
  for (int k = 0; k < 4; ++k) dq[k] = (gq[k] - dot * G->qhat[k]) / G->qnorm;
}

/* ---------------------------------------------------------------------------------------------
 * Backward (§3.3 gradient equations).  I, W, gI: [nz][ny][nx] (forward outputs and dL/dI).
 * sel: optional list of Gaussian indices (NULL: all).  Gradients are written at the Gaussian's
 * own index in the n-sized outputs; entries not selected are left untouched.  d_relax may be NULL.
 */
int og_grad(int64_t n, const float *mu, const float *log_scale, const float *quat, const float *amp,
            const float *relax, int nx, int ny, int nz, const double *origin, const double *spacing, double cutoff,
            double eps, const double *I, const double *W, const double *gI, int64_t nsel, const int64_t *sel,
            double *d_mu, double *d_log_scale, double *d_quat, double *d_amp, double *d_relax, int nthreads) {
  og_grid_t g;
  make_grid(&g, nx, ny, nz, origin, spacing);
  int64_t m = sel ? nsel : n;
  int bad = 0;
  real_t c2 = (real_t)cutoff * (real_t)cutoff;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 16) reduction(| : bad)
  for (int64_t k = 0; k < m; ++k) {
    int64_t i = sel ? sel[k] : k;
    og_gauss_t Gi;
    if (i < 0 || i >= n || setup_gauss(&Gi, i, mu, log_scale, quat, amp, relax, &g, (real_t)cutoff) != 0) {
      bad = 1;
      continue;
    }
    real_t dA = 0, dr = 0, sk[3] = {0, 0, 0}, M[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    if (!(Gi.lo[0] > Gi.hi[0] || Gi.lo[1] > Gi.hi[1] || Gi.lo[2] > Gi.hi[2])) {
      for (int iz = Gi.lo[2]; iz <= Gi.hi[2]; ++iz)
        for (int iy = Gi.lo[1]; iy <= Gi.hi[1]; ++iy)
          for (int ix = Gi.lo[0]; ix <= Gi.hi[0]; ++ix) {
            real_t d[3];
            real_t d2 = maha2(&Gi, &g, ix, iy, iz, d);
            if (!(d2 <= c2)) continue;
            int64_t v = vidx(&g, ix, iy, iz);
            real_t Gval = R_EXP(-d2 / 2);
            real_t w = Gi.r * Gval;
            real_t cp = (real_t)gI[v] / ((real_t)W[v] + (real_t)eps); /* dL/dI / (W + eps) */
            real_t e = cp * (Gi.A - (real_t)I[v]);                     /* dL/dw_i(p) */
            dA += cp * w;
            dr += e * Gval;
            real_t kappa = e * w;
            for (int a = 0; a < 3; ++a) {
              sk[a] += kappa * d[a];
              for (int b = 0; b < 3; ++b) M[a][b] += kappa * d[a] * d[b];
            }
          }
    }
    /* dL/dmu = P sum(kappa delta);  dL/dP = -1/2 sum(kappa delta delta^T) */
    real_t Gp[3][3], ds[3], dq[4];
    for (int a = 0; a < 3; ++a) {
      real_t s = 0;
      for (int b = 0; b < 3; ++b) {
        s += Gi.P[a][b] * sk[b];
        Gp[a][b] = -M[a][b] / 2;
      }
      d_mu[3 * i + a] = (double)s;
    }
    chain_to_scale_quat(&Gi, Gp, ds, dq);
    for (int a = 0; a < 3; ++a) d_log_scale[3 * i + a] = (double)ds[a];
    for (int a = 0; a < 4; ++a) d_quat[4 * i + a] = (double)dq[a];
    d_amp[i] = (double)dA;
    if (d_relax) d_relax[i] = (double)dr;
  }
  return bad ? -1 : 0;
}

/* ---------------------------------------------------------------------------------------------
 * Counting helpers for measurement and for conditioning parity inputs.
 */

/* Number of useful pairs (voxel, Gaussian) with d^2 <= cutoff^2 on the grid. */
int64_t og_count_pairs(int64_t n, const float *mu, const float *log_scale, const float *quat, int nx, int ny, int nz,
                       const double *origin, const double *spacing, double cutoff, int nthreads) {
  og_grid_t g;
  make_grid(&g, nx, ny, nz, origin, spacing);
  float one = 1;
  real_t c2 = (real_t)cutoff * (real_t)cutoff;
  int64_t total = 0;
  int bad = 0;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 64) reduction(+ : total) reduction(| : bad)
  for (int64_t i = 0; i < n; ++i) {
    og_gauss_t Gi;
    float a1 = one;
    if (setup_gauss(&Gi, 0, mu + 3 * i, log_scale + 3 * i, quat + 4 * i, &a1, NULL, &g, (real_t)cutoff) != 0) {
      bad = 1;
      continue;
    }
    if (Gi.lo[0] > Gi.hi[0] || Gi.lo[1] > Gi.hi[1] || Gi.lo[2] > Gi.hi[2]) continue;
    for (int iz = Gi.lo[2]; iz <= Gi.hi[2]; ++iz)
      for (int iy = Gi.lo[1]; iy <= Gi.hi[1]; ++iy)
        for (int ix = Gi.lo[0]; ix <= Gi.hi[0]; ++ix) {
          real_t d[3];
          if (maha2(&Gi, &g, ix, iy, iz, d) <= c2) ++total;
        }
  }
  return bad ? -1 : total;
}

/* Per Gaussian, the number of voxels whose d^2 lies within `band` of cutoff^2 (pairs whose
 * inclusion can legitimately differ between FP32 and FP64 evaluation).  sel: optional subset. */
int og_ambiguous(int64_t n, const float *mu, const float *log_scale, const float *quat, int nx, int ny, int nz,
                 const double *origin, const double *spacing, double cutoff, double band, int64_t nsel,
                 const int64_t *sel, int32_t *count, int nthreads) {
  og_grid_t g;
  make_grid(&g, nx, ny, nz, origin, spacing);
  int64_t m = sel ? nsel : n;
  real_t c2 = (real_t)cutoff * (real_t)cutoff;
  int bad = 0;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 64) reduction(| : bad)
  for (int64_t k = 0; k < m; ++k) {
    int64_t i = sel ? sel[k] : k;
    og_gauss_t Gi;
    float a1 = 1;
    /* widen the box so that pairs just outside the cutoff are seen too */
    if (i < 0 || i >= n ||
        setup_gauss(&Gi, 0, mu + 3 * i, log_scale + 3 * i, quat + 4 * i, &a1, NULL, &g,
                    R_SQRT(c2 + (real_t)band)) != 0) {
      bad = 1;
      continue;
    }
    int32_t c = 0;
    if (!(Gi.lo[0] > Gi.hi[0] || Gi.lo[1] > Gi.hi[1] || Gi.lo[2] > Gi.hi[2]))
      for (int iz = Gi.lo[2]; iz <= Gi.hi[2]; ++iz)
        for (int iy = Gi.lo[1]; iy <= Gi.hi[1]; ++iy)
          for (int ix = Gi.lo[0]; ix <= Gi.hi[0]; ++ix) {
            real_t d[3];
            if (R_FABS(maha2(&Gi, &g, ix, iy, iz, d) - c2) <= (real_t)band) ++c;
          }
    count[k] = c;
  }
  return bad ? -1 : 0;
}

/* Index box of each Gaussian (inclusive lo/hi per axis, [n][6] = lo x,y,z, hi x,y,z). */
int og_index_boxes(int64_t n, const float *mu, const float *log_scale, const float *quat, int nx, int ny, int nz,
                   const double *origin, const double *spacing, double cutoff, int32_t *box) {
  og_grid_t g;
  make_grid(&g, nx, ny, nz, origin, spacing);
  float one = 1;
  for (int64_t i = 0; i < n; ++i) {
    og_gauss_t Gi;
    if (setup_gauss(&Gi, 0, mu + 3 * i, log_scale + 3 * i, quat + 4 * i, &one, NULL, &g, (real_t)cutoff) != 0)
      return -1;
    for (int k = 0; k < 3; ++k) {
      box[6 * i + k] = Gi.lo[k];
      box[6 * i + 3 + k] = Gi.hi[k];
    }
  }
  return 0;
}

/* ---------------------------------------------------------------------------------------------
 * Forward with the support held fixed: the pair (p, i) is kept iff its d^2 under a second
 * parameter set (mu0, log_scale0, quat0) is <= cutoff^2, and weighted with the first set.  The
 * analytic gradient of §3.3 is the derivative of this function at (mu0, ...) = (mu, ...), which is
 * what central differences of it measure.
 */
int og_render_frozen(int64_t n, const float *mu, const float *log_scale, const float *quat, const float *amp,
                     const float *relax, const float *mu0, const float *log_scale0, const float *quat0, int nx,
                     int ny, int nz, const double *origin, const double *spacing, double cutoff, double eps,
                     double *I, double *W, int nthreads) {
  og_grid_t g;
  make_grid(&g, nx, ny, nz, origin, spacing);
  int64_t V = (int64_t)nx * ny * nz;
  og_gauss_t *G = (og_gauss_t *)malloc(sizeof(og_gauss_t) * (size_t)(n > 0 ? n : 1));
  og_gauss_t *G0 = (og_gauss_t *)malloc(sizeof(og_gauss_t) * (size_t)(n > 0 ? n : 1));
  real_t *Wacc = (real_t *)calloc((size_t)V, sizeof(real_t));
  real_t *Sacc = (real_t *)calloc((size_t)V, sizeof(real_t));
  if (!G || !G0 || !Wacc || !Sacc) {
    free(G);
    free(G0);
    free(Wacc);
    free(Sacc);
    return -2;
  }
  int rc = setup_all(G, n, mu, log_scale, quat, amp, relax, &g, (real_t)cutoff, nthreads);
  if (rc == 0) rc = setup_all(G0, n, mu0, log_scale0, quat0, amp, relax, &g, (real_t)cutoff, nthreads);
  real_t c2 = (real_t)cutoff * (real_t)cutoff;
  if (rc == 0) {
#pragma omp parallel num_threads(nthreads)
    {
      int T = omp_get_num_threads(), t = omp_get_thread_num();
      int z0 = (int)((int64_t)nz * t / T), z1 = (int)((int64_t)nz * (t + 1) / T);
      for (int64_t i = 0; i < n; ++i) {
        const og_gauss_t *Gs = &G0[i], *Gw = &G[i];
        if (Gs->lo[0] > Gs->hi[0] || Gs->lo[1] > Gs->hi[1] || Gs->lo[2] > Gs->hi[2]) continue;
        int za = Gs->lo[2] > z0 ? Gs->lo[2] : z0;
        int zb = Gs->hi[2] < z1 - 1 ? Gs->hi[2] : z1 - 1;
        for (int iz = za; iz <= zb; ++iz)
          for (int iy = Gs->lo[1]; iy <= Gs->hi[1]; ++iy)
            for (int ix = Gs->lo[0]; ix <= Gs->hi[0]; ++ix) {
              real_t d[3];
              if (maha2(Gs, &g, ix, iy, iz, d) <= c2) {
                real_t w = Gw->r * R_EXP(-maha2(Gw, &g, ix, iy, iz, d) / 2);
                int64_t v = vidx(&g, ix, iy, iz);
                Wacc[v] += w;
                Sacc[v] += Gw->A * w;
              }
            }
      }
    }
    for (int64_t v = 0; v < V; ++v) {
      I[v] = (double)(Sacc[v] / (Wacc[v] + (real_t)eps));
      if (W) W[v] = (double)Wacc[v];
    }
  }
  free(G);
  free(G0);
  free(Wacc);
  free(Sacc);
  return rc;
}

/* Per voxel, the number of Gaussians whose d^2 at that voxel lies within `band` of cutoff^2 (the
 * voxels whose value depends on an inclusion decision that FP32 and FP64 may take differently). */
int og_ambiguous_voxels(int64_t n, const float *mu, const float *log_scale, const float *quat, int nx, int ny, int nz,
                        const double *origin, const double *spacing, double cutoff, double band, int32_t *count,
                        int nthreads) {
  og_grid_t g;
  make_grid(&g, nx, ny, nz, origin, spacing);
  og_gauss_t *G = (og_gauss_t *)malloc(sizeof(og_gauss_t) * (size_t)(n > 0 ? n : 1));
  if (!G) return -2;
  real_t c2 = (real_t)cutoff * (real_t)cutoff;
  real_t cw = R_SQRT(c2 + (real_t)band);
  float one = 1;
  int bad = 0;
#pragma omp parallel for num_threads(nthreads) schedule(static) reduction(| : bad)
  for (int64_t i = 0; i < n; ++i) {
    float a1 = one;
    bad |= setup_gauss(&G[i], 0, mu + 3 * i, log_scale + 3 * i, quat + 4 * i, &a1, NULL, &g, cw) != 0;
  }
  if (bad) {
    free(G);
    return -1;
  }
  memset(count, 0, sizeof(int32_t) * (size_t)nx * ny * nz);
#pragma omp parallel num_threads(nthreads)
  {
    int T = omp_get_num_threads(), t = omp_get_thread_num();
    int z0 = (int)((int64_t)nz * t / T), z1 = (int)((int64_t)nz * (t + 1) / T);
    for (int64_t i = 0; i < n; ++i) {
      const og_gauss_t *Gi = &G[i];
      if (Gi->lo[0] > Gi->hi[0] || Gi->lo[1] > Gi->hi[1] || Gi->lo[2] > Gi->hi[2]) continue;
      int za = Gi->lo[2] > z0 ? Gi->lo[2] : z0;
      int zb = Gi->hi[2] < z1 - 1 ? Gi->hi[2] : z1 - 1;
      for (int iz = za; iz <= zb; ++iz)
        for (int iy = Gi->lo[1]; iy <= Gi->hi[1]; ++iy)
          for (int ix = Gi->lo[0]; ix <= Gi->hi[0]; ++ix) {
            real_t d[3];
            if (R_FABS(maha2(Gi, &g, ix, iy, iz, d) - c2) <= (real_t)band) count[vidx(&g, ix, iy, iz)] += 1;
          }
    }
  }
  free(G);
  return 0;
}
