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
#include <float.h>
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

/* ---------------------------------------------------------------------------------------------
 * A-priori rounding-error bounds of this oracle's own arithmetic, per output entry (the FP64
 * oracle error; the same code bounds the long double build with its own unit roundoff).
 *
 * u is the unit roundoff of real_t and gam(k) = k u / (1 - k u), the classical bound on the
 * relative error of k successive roundings (a recursive sum of k + 1 terms, or a product chain).
 *
 * One pair (voxel p, Gaussian i).  The computed delta_a = (o_a + h_a i_a) - mu_a is within
 * e_a = 3 u (|o_a| + |h_a i_a| + |mu_a|) of the exact one.  The computed P = R diag(D) R^T,
 * D_k = exp(-2 s_k), is within gam(5) Pabs + 40 u Dmax of the exact one entrywise, where
 * Pabs = |R| diag(D) |R|^T >= |P| and Dmax = max_k D_k (the rotation entries come from the
 * normalised quaternion within about 8 u absolute each, |R| <= 1; exp within one ulp).  The
 * quadratic form sums 9 terms of two products each.  Hence the computed d^2 is within
 *   D2 = gam(30) |delta|^T Pabs |delta| + 40 u Dmax (sum_a |delta_a|)^2 + 2 e^T Pabs |delta|
 * of the exact d^2, and the weight w = r exp(-d^2 / 2) has relative error at most
 *   tau = 0.505 D2 + 3 u      (exp and the product with r within one ulp each),
 * provided the pair is decided as the exact arithmetic decides it, i.e. |d^2 - cutoff^2| > D2.
 * The functions below report the smallest |d^2 - cutoff^2| - D2 over every pair of every box they
 * visit (min_margin) so that this precondition can be checked.
 */
#ifdef OG_LONG_DOUBLE
#define OG_U ((real_t)LDBL_EPSILON / 2)
#else
#define OG_U ((real_t)DBL_EPSILON / 2)
#endif

static real_t gam(real_t k) { return k * OG_U / (1 - k * OG_U); }

/* Pabs and Dmax of a Gaussian (see above). */
static void abs_frame(const og_gauss_t *G, real_t Pabs[3][3], real_t *Dmax) {
  real_t D[3];
  *Dmax = 0;
  for (int k = 0; k < 3; ++k) {
    D[k] = 1 / G->ev[k];
    if (D[k] > *Dmax) *Dmax = D[k];
  }
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      real_t s = 0;
      for (int k = 0; k < 3; ++k) s += R_FABS(G->R[a][k]) * D[k] * R_FABS(G->R[b][k]);
      Pabs[a][b] = s;
    }
}

/* D2 of the pair (see above); e receives the error bound of each delta entry. */
static real_t pair_d2_err(const og_gauss_t *G, const og_grid_t *g, const real_t Pabs[3][3], real_t Dmax, int ix,
                          int iy, int iz, const real_t d[3], real_t e[3]) {
  const int idx[3] = {ix, iy, iz};
  real_t ad[3], l1 = 0;
  for (int a = 0; a < 3; ++a) {
    ad[a] = R_FABS(d[a]);
    l1 += ad[a];
    e[a] = 3 * OG_U * (R_FABS(g->o[a]) + R_FABS(g->h[a] * idx[a]) + R_FABS(G->mu[a]));
  }
  real_t quad = 0, lin = 0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      quad += ad[a] * Pabs[a][b] * ad[b];
      lin += e[a] * Pabs[a][b] * ad[b];
    }
  return gam(30) * quad + 40 * OG_U * Dmax * l1 * l1 + 2 * lin;
}

/* Error bound of the forward at every voxel: |I_computed - I_exact| <= bI, likewise bW, for the
 * truncated sums of og_render (each voxel: W = sum of K weights with relative errors <= tau,
 * summed recursively; S = sum of A w; I = S / (W + eps)):
 *   bW = (tau + gam(K) (1 + tau)) W,    bS = (tau + u + gam(K) (1 + tau + u)) sum |A w|,
 *   bI = (bS + |I| bW) / (W + eps) + 2 u |I|          (the addition of eps and the division),
 * all times (1 + 1e-9) for the second-order terms.  *min_margin: see above. */
int og_render_bound(int64_t n, const float *mu, const float *log_scale, const float *quat, const float *amp,
                    const float *relax, int nx, int ny, int nz, const double *origin, const double *spacing,
                    double cutoff, double eps, double *bI, double *bW, double *min_margin, int nthreads) {
  og_grid_t g;
  make_grid(&g, nx, ny, nz, origin, spacing);
  int64_t V = (int64_t)nx * ny * nz;
  og_gauss_t *G = (og_gauss_t *)malloc(sizeof(og_gauss_t) * (size_t)(n > 0 ? n : 1));
  real_t *Wa = (real_t *)calloc((size_t)V, sizeof(real_t));
  real_t *Sa = (real_t *)calloc((size_t)V, sizeof(real_t));
  real_t *Sabs = (real_t *)calloc((size_t)V, sizeof(real_t));
  real_t *tau = (real_t *)calloc((size_t)V, sizeof(real_t));
  int32_t *K = (int32_t *)calloc((size_t)V, sizeof(int32_t));
  if (!G || !Wa || !Sa || !Sabs || !tau || !K) {
    free(G); free(Wa); free(Sa); free(Sabs); free(tau); free(K);
    return -2;
  }
  int rc = setup_all(G, n, mu, log_scale, quat, amp, relax, &g, (real_t)cutoff, nthreads);
  real_t c2 = (real_t)cutoff * (real_t)cutoff;
  real_t margin = INFINITY;
  if (rc == 0) {
#pragma omp parallel num_threads(nthreads) reduction(min : margin)
    {
      int T = omp_get_num_threads(), t = omp_get_thread_num();
      int z0 = (int)((int64_t)nz * t / T), z1 = (int)((int64_t)nz * (t + 1) / T);
      for (int64_t i = 0; i < n; ++i) {
        const og_gauss_t *Gi = &G[i];
        if (Gi->lo[0] > Gi->hi[0] || Gi->lo[1] > Gi->hi[1] || Gi->lo[2] > Gi->hi[2]) continue;
        int za = Gi->lo[2] > z0 ? Gi->lo[2] : z0;
        int zb = Gi->hi[2] < z1 - 1 ? Gi->hi[2] : z1 - 1;
        if (za > zb) continue;
        real_t Pabs[3][3], Dmax;
        abs_frame(Gi, Pabs, &Dmax);
        for (int iz = za; iz <= zb; ++iz)
          for (int iy = Gi->lo[1]; iy <= Gi->hi[1]; ++iy)
            for (int ix = Gi->lo[0]; ix <= Gi->hi[0]; ++ix) {
              real_t d[3], e[3];
              real_t d2 = maha2(Gi, &g, ix, iy, iz, d);
              real_t D2 = pair_d2_err(Gi, &g, Pabs, Dmax, ix, iy, iz, d, e);
              real_t m = R_FABS(d2 - c2) - D2;
              if (m < margin) margin = m;
              if (d2 <= c2) {
                real_t w = Gi->r * R_EXP(-d2 / 2);
                int64_t v = vidx(&g, ix, iy, iz);
                real_t tp = (real_t)0.505 * D2 + 3 * OG_U;
                Wa[v] += w;
                Sa[v] += Gi->A * w;
                Sabs[v] += R_FABS(Gi->A * w);
                if (tp > tau[v]) tau[v] = tp;
                K[v] += 1;
              }
            }
      }
    }
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t v = 0; v < V; ++v) {
      real_t gk = gam((real_t)K[v]), tv = tau[v];
      real_t bw = (tv + gk * (1 + tv)) * Wa[v];
      real_t bs = (tv + OG_U + gk * (1 + tv + OG_U)) * Sabs[v];
      real_t I = Sa[v] / (Wa[v] + (real_t)eps);
      real_t bi = (bs + R_FABS(I) * bw) / (Wa[v] + (real_t)eps) + 2 * OG_U * R_FABS(I);
      bW[v] = (double)(bw * (1 + (real_t)1e-9));
      bI[v] = (double)(bi * (1 + (real_t)1e-9));
    }
  }
  if (min_margin) *min_margin = (double)margin;
  free(G); free(Wa); free(Sa); free(Sabs); free(tau); free(K);
  return rc;
}

/* |J| x for the chain rule of og_grad (from the brick sums to d_mu, d_log_scale, d_quat), with
 * every signed quantity replaced by its magnitude (and the rotation entries by |R| + 16 u, which
 * covers their own rounding): an upper bound of the map's absolute value applied to the nonnegative
 * vector x = (x_sk[3], x_M[3][3]).  out: d_mu 3, d_log_scale 3, d_quat 4. */
static void chain_abs(const og_gauss_t *G, const real_t xsk[3], const real_t xM[3][3], real_t out[10]) {
  real_t Ra[3][3], D[3], Pa[3][3], qa[4];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) Ra[a][b] = R_FABS(G->R[a][b]) + 16 * OG_U;
  for (int k = 0; k < 3; ++k) D[k] = 1 / G->ev[k];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      real_t s = 0;
      for (int k = 0; k < 3; ++k) s += Ra[a][k] * D[k] * Ra[b][k];
      Pa[a][b] = s;
    }
  for (int k = 0; k < 4; ++k) qa[k] = R_FABS(G->qhat[k]) + 4 * OG_U;
  for (int a = 0; a < 3; ++a) {
    real_t s = 0;
    for (int b = 0; b < 3; ++b) s += Pa[a][b] * xsk[b];
    out[a] = s;
  }
  real_t xG[3][3], dR[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) xG[a][b] = xM[a][b] / 2;
  for (int k = 0; k < 3; ++k) {
    real_t s = 0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) s += Ra[a][k] * xG[a][b] * Ra[b][k];
    out[3 + k] = 2 * D[k] * s;
  }
  for (int a = 0; a < 3; ++a)
    for (int k = 0; k < 3; ++k) {
      real_t s = 0;
      for (int b = 0; b < 3; ++b) s += xG[a][b] * Ra[b][k];
      dR[a][k] = 2 * s * D[k];
    }
  real_t w = qa[0], x = qa[1], y = qa[2], z = qa[3];
  real_t gw = 2 * (z * dR[0][1] + y * dR[0][2] + z * dR[1][0] + x * dR[1][2] + y * dR[2][0] + x * dR[2][1]);
  real_t gx = 2 * (y * dR[0][1] + z * dR[0][2] + y * dR[1][0] + 2 * x * dR[1][1] + w * dR[1][2] + z * dR[2][0] +
                   w * dR[2][1] + 2 * x * dR[2][2]);
  real_t gy = 2 * (2 * y * dR[0][0] + x * dR[0][1] + w * dR[0][2] + x * dR[1][0] + z * dR[1][2] + w * dR[2][0] +
                   z * dR[2][1] + 2 * y * dR[2][2]);
  real_t gz = 2 * (2 * z * dR[0][0] + w * dR[0][1] + x * dR[0][2] + w * dR[1][0] + 2 * z * dR[1][1] +
                   y * dR[1][2] + x * dR[2][0] + y * dR[2][1]);
  real_t gq[4] = {gw, gx, gy, gz};
  real_t dot = 0;
  for (int k = 0; k < 4; ++k) dot += qa[k] * gq[k];
  for (int k = 0; k < 4; ++k) out[6 + k] = (gq[k] + dot * qa[k]) / G->qnorm;
}

/* Error bound of og_grad's outputs for the selected Gaussians (the stage-wise gradient: I, W and
 * dL/dI given exactly as doubles).  Per pair, the terms of the 11 sums and their relative errors:
 *   cp = gI / (W + eps) (2 u), G = exp(-d^2/2) (0.505 D2 + 2 u), w = r G (+ u),
 *   e = cp (A - I) (+ 2 u), kappa = e w (+ u); terms cp w, e G, kappa delta_a (+ u, and |kappa| e_a
 *   from delta), kappa delta_a delta_b (+ 2 u, and |kappa| (e_a |delta_b| + |delta_a| e_b)).
 * For each sum j: A_j = sum |t| and E_j = sum |dt| over its K terms; its error is at most
 * B_j = E_j + gam(K) (A_j + E_j).  The chain rule (from the sums to the parameters) is linear in the
 * sums with coefficients made of R, D and the normalised quaternion; its output error is at most
 * |J| B + gam(60) |J| (A + B) (the second term: the chain's own roundings), with |J| as in
 * chain_abs.  bound: [n][12] per Gaussian, in the order d_mu 3, d_log_scale 3, d_quat 4, d_amp,
 * d_relax; rows not selected are left untouched.  *min_margin: see above. */
int og_grad_bound(int64_t n, const float *mu, const float *log_scale, const float *quat, const float *amp,
                  const float *relax, int nx, int ny, int nz, const double *origin, const double *spacing,
                  double cutoff, double eps, const double *I, const double *W, const double *gI, int64_t nsel,
                  const int64_t *sel, double *bound, double *min_margin, int nthreads) {
  og_grid_t g;
  make_grid(&g, nx, ny, nz, origin, spacing);
  int64_t m = sel ? nsel : n;
  int bad = 0;
  real_t c2 = (real_t)cutoff * (real_t)cutoff;
  real_t margin = INFINITY;
  const real_t u = OG_U;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 16) reduction(| : bad) reduction(min : margin)
  for (int64_t k = 0; k < m; ++k) {
    int64_t i = sel ? sel[k] : k;
    og_gauss_t Gi;
    if (i < 0 || i >= n || setup_gauss(&Gi, i, mu, log_scale, quat, amp, relax, &g, (real_t)cutoff) != 0) {
      bad = 1;
      continue;
    }
    real_t Pabs[3][3], Dmax;
    abs_frame(&Gi, Pabs, &Dmax);
    /* sums: 0 = dA, 1 = dr, 2..4 = kappa delta, 5..13 = kappa delta delta^T (3 x 3, row-major) */
    real_t As[14], Es[14];
    for (int j = 0; j < 14; ++j) As[j] = Es[j] = 0;
    int64_t K = 0;
    if (!(Gi.lo[0] > Gi.hi[0] || Gi.lo[1] > Gi.hi[1] || Gi.lo[2] > Gi.hi[2])) {
      for (int iz = Gi.lo[2]; iz <= Gi.hi[2]; ++iz)
        for (int iy = Gi.lo[1]; iy <= Gi.hi[1]; ++iy)
          for (int ix = Gi.lo[0]; ix <= Gi.hi[0]; ++ix) {
            real_t d[3], e[3];
            real_t d2 = maha2(&Gi, &g, ix, iy, iz, d);
            real_t D2 = pair_d2_err(&Gi, &g, Pabs, Dmax, ix, iy, iz, d, e);
            real_t mg = R_FABS(d2 - c2) - D2;
            if (mg < margin) margin = mg;
            if (!(d2 <= c2)) continue;
            ++K;
            int64_t v = vidx(&g, ix, iy, iz);
            real_t Gv = R_EXP(-d2 / 2);
            real_t w = Gi.r * Gv;
            real_t cp = (real_t)gI[v] / ((real_t)W[v] + (real_t)eps);
            real_t ee = cp * (Gi.A - (real_t)I[v]);
            real_t kap = ee * w;
            real_t tG = (real_t)0.505 * D2 + 2 * u;
            real_t rA = 2 * u + tG + u + u;          /* cp w */
            real_t rr = 4 * u + tG + u;              /* e G */
            real_t rk = 4 * u + tG + u + u;          /* kappa */
            real_t t;
            t = R_FABS(cp * w);
            As[0] += t;
            Es[0] += rA * t;
            t = R_FABS(ee * Gv);
            As[1] += t;
            Es[1] += rr * t;
            for (int a = 0; a < 3; ++a) {
              t = R_FABS(kap * d[a]);
              As[2 + a] += t;
              Es[2 + a] += (rk + u) * t + R_FABS(kap) * e[a];
              for (int b = 0; b < 3; ++b) {
                t = R_FABS(kap * d[a] * d[b]);
                As[5 + 3 * a + b] += t;
                Es[5 + 3 * a + b] += (rk + 2 * u) * t + R_FABS(kap) * (e[a] * R_FABS(d[b]) + R_FABS(d[a]) * e[b]);
              }
            }
          }
    }
    real_t gk = gam((real_t)K);
    real_t B[14], AB[14];
    for (int j = 0; j < 14; ++j) {
      B[j] = Es[j] + gk * (As[j] + Es[j]);
      AB[j] = As[j] + B[j];
    }
    real_t oB[10], oAB[10];
    real_t xM[3][3], xMA[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        xM[a][b] = B[5 + 3 * a + b];
        xMA[a][b] = AB[5 + 3 * a + b];
      }
    chain_abs(&Gi, B + 2, xM, oB);
    chain_abs(&Gi, AB + 2, xMA, oAB);
    real_t gc = gam(60);
    for (int j = 0; j < 10; ++j) bound[12 * i + j] = (double)((oB[j] + gc * oAB[j]) * (1 + (real_t)1e-9));
    bound[12 * i + 10] = (double)(B[0] * (1 + (real_t)1e-9));
    bound[12 * i + 11] = (double)(B[1] * (1 + (real_t)1e-9));
  }
  if (min_margin) *min_margin = (double)margin;
  return bad ? -1 : 0;
}

/* ---------------------------------------------------------------------------------------------
 * Forward with the inclusion of every ambiguous pair left open.  A pair with
 * |d^2 - cutoff^2| <= band may be included or excluded (an FP32 and an FP64 evaluation of d^2 can
 * disagree there, and both are correct readings of the 3-sigma truncation).  Per voxel with k such
 * pairs (k <= maxk), Ilo/Ihi and Wlo/Whi receive the minimum and maximum of I and W over all 2^k
 * include/exclude choices, the other pairs being decided as og_render decides them; voxels with no
 * ambiguous pair get lo = hi = og_render's value; voxels with k > maxk get lo = -inf, hi = +inf.
 * namb (may be NULL) receives k per voxel.  Returns the number of voxels with k > maxk, or a
 * negative code. */
int64_t og_render_envelope(int64_t n, const float *mu, const float *log_scale, const float *quat, const float *amp,
                           const float *relax, int nx, int ny, int nz, const double *origin, const double *spacing,
                           double cutoff, double eps, double band, int maxk, double *Ilo, double *Ihi, double *Wlo,
                           double *Whi, int32_t *namb, int nthreads) {
  og_grid_t g;
  make_grid(&g, nx, ny, nz, origin, spacing);
  int64_t V = (int64_t)nx * ny * nz;
  real_t c2 = (real_t)cutoff * (real_t)cutoff, bd = (real_t)band;
  og_gauss_t *G = (og_gauss_t *)malloc(sizeof(og_gauss_t) * (size_t)(n > 0 ? n : 1));
  real_t *W0 = (real_t *)calloc((size_t)V, sizeof(real_t));
  real_t *S0 = (real_t *)calloc((size_t)V, sizeof(real_t));
  int32_t *cnt = (int32_t *)calloc((size_t)V, sizeof(int32_t));
  int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)(V + 1));
  if (!G || !W0 || !S0 || !cnt || !start) {
    free(G); free(W0); free(S0); free(cnt); free(start);
    return -2;
  }
  /* the index box is widened so that pairs just outside the cutoff are seen */
  int rc = setup_all(G, n, mu, log_scale, quat, amp, relax, &g, R_SQRT(c2 + bd), nthreads);
  if (rc != 0) {
    free(G); free(W0); free(S0); free(cnt); free(start);
    return rc;
  }
  /* pass 1: the sums over the decided pairs, and the number of open pairs per voxel */
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
            real_t d2 = maha2(Gi, &g, ix, iy, iz, d);
            int64_t v = vidx(&g, ix, iy, iz);
            if (R_FABS(d2 - c2) <= bd) {
              cnt[v] += 1;
            } else if (d2 <= c2) {
              real_t w = Gi->r * R_EXP(-d2 / 2);
              W0[v] += w;
              S0[v] += Gi->A * w;
            }
          }
    }
  }
  start[0] = 0;
  for (int64_t v = 0; v < V; ++v) start[v + 1] = start[v] + cnt[v];
  int64_t total = start[V];
  real_t *pw = (real_t *)malloc(sizeof(real_t) * (size_t)(total > 0 ? total : 1));
  real_t *ps = (real_t *)malloc(sizeof(real_t) * (size_t)(total > 0 ? total : 1));
  int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)(V > 0 ? V : 1));
  if (!pw || !ps || !cur) {
    free(G); free(W0); free(S0); free(cnt); free(start); free(pw); free(ps); free(cur);
    return -2;
  }
  memcpy(cur, start, sizeof(int64_t) * (size_t)V);
  /* pass 2: the open pairs' weights, per voxel in ascending Gaussian order */
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
            real_t d2 = maha2(Gi, &g, ix, iy, iz, d);
            if (R_FABS(d2 - c2) <= bd) {
              int64_t v = vidx(&g, ix, iy, iz);
              real_t w = Gi->r * R_EXP(-d2 / 2);
              pw[cur[v]] = w;
              ps[cur[v]] = Gi->A * w;
              cur[v] += 1;
            }
          }
    }
  }
  /* pass 3: extremes over the include/exclude choices */
  int64_t skipped = 0;
#pragma omp parallel for num_threads(nthreads) schedule(static) reduction(+ : skipped)
  for (int64_t v = 0; v < V; ++v) {
    int k = cnt[v];
    if (namb) namb[v] = k;
    if (k > maxk) {
      Ilo[v] = Wlo[v] = -INFINITY;
      Ihi[v] = Whi[v] = INFINITY;
      ++skipped;
      continue;
    }
    real_t ilo = INFINITY, ihi = -INFINITY, wlo = INFINITY, whi = -INFINITY;
    for (int64_t mask = 0; mask < ((int64_t)1 << k); ++mask) {
      real_t Wv = W0[v], Sv = S0[v];
      for (int j = 0; j < k; ++j)
        if ((mask >> j) & 1) {
          Wv += pw[start[v] + j];
          Sv += ps[start[v] + j];
        }
      real_t Iv = Sv / (Wv + (real_t)eps);
      if (Iv < ilo) ilo = Iv;
      if (Iv > ihi) ihi = Iv;
      if (Wv < wlo) wlo = Wv;
      if (Wv > whi) whi = Wv;
    }
    Ilo[v] = (double)ilo;
    Ihi[v] = (double)ihi;
    Wlo[v] = (double)wlo;
    Whi[v] = (double)whi;
  }
  free(G); free(W0); free(S0); free(cnt); free(start); free(pw); free(ps); free(cur);
  return skipped;
}

/* ---------------------------------------------------------------------------------------------
 * Weights of one Gaussian with its support held fixed, over the padded index box of the support:
 * the Gaussian (mu, log_scale, quat, amp, relax; one entry each) is weighed as in og_render, and
 * the pair predicate d^2 <= cutoff^2 is taken with a second parameter set (mu0, log_scale0, quat0;
 * one entry each) whose box is used.  Writes box[6] = (lo x, y, z, hi x, y, z) of that box and, if
 * vox and w are not NULL and cap is at least the box's voxel count, the flat index (x fastest) and
 * the weight (0 for a pair outside the support) of every box voxel in x-fastest order.  Returns the
 * box's voxel count, or -1 for an invalid input.  (Finite differences of the loss in one parameter
 * of one Gaussian change only these voxels.) */
int64_t og_weights_box(const float *mu, const float *log_scale, const float *quat, const float *amp,
                       const float *relax, const float *mu0, const float *log_scale0, const float *quat0, int nx,
                       int ny, int nz, const double *origin, const double *spacing, double cutoff, int32_t *box,
                       int64_t cap, int64_t *vox, double *w) {
  og_grid_t g;
  make_grid(&g, nx, ny, nz, origin, spacing);
  og_gauss_t Gw, Gs;
  float one = 1;
  if (setup_gauss(&Gw, 0, mu, log_scale, quat, amp, relax, &g, (real_t)cutoff) != 0) return -1;
  if (setup_gauss(&Gs, 0, mu0, log_scale0, quat0, &one, NULL, &g, (real_t)cutoff) != 0) return -1;
  for (int k = 0; k < 3; ++k) {
    box[k] = Gs.lo[k];
    box[3 + k] = Gs.hi[k];
  }
  if (Gs.lo[0] > Gs.hi[0] || Gs.lo[1] > Gs.hi[1] || Gs.lo[2] > Gs.hi[2]) return 0;
  int64_t cnt = (int64_t)(Gs.hi[0] - Gs.lo[0] + 1) * (Gs.hi[1] - Gs.lo[1] + 1) * (Gs.hi[2] - Gs.lo[2] + 1);
  if (!vox || !w || cap < cnt) return cnt;
  real_t c2 = (real_t)cutoff * (real_t)cutoff;
  int64_t k = 0;
  for (int iz = Gs.lo[2]; iz <= Gs.hi[2]; ++iz)
    for (int iy = Gs.lo[1]; iy <= Gs.hi[1]; ++iy)
      for (int ix = Gs.lo[0]; ix <= Gs.hi[0]; ++ix) {
        real_t d[3];
        vox[k] = vidx(&g, ix, iy, iz);
        w[k] = maha2(&Gs, &g, ix, iy, iz, d) <= c2 ? (double)(Gw.r * R_EXP(-maha2(&Gw, &g, ix, iy, iz, d) / 2)) : 0.0;
        ++k;
      }
  return cnt;
}
