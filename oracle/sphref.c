/*
 * sphref.c -- plain FP64 CPU oracle of the feature-aware SPH relaxation step.
 *
 * TEST INFRASTRUCTURE ONLY (see sphref.h): used by the tests, the smoke check
 * and the benchmark's CPU baseline; never by the GPU product path.
 *
 * The code follows the paper section by section:
 *   geometry and features ........ sec. 3.1-3.2 (level set, feature tags,
 *                                   particle types P_si, P_c, P_s, P_+)
 *   target feature size .......... sec. 2.2, Eq. (target_mesh_gen)
 *   kernel ....................... Wendland C2 reaching r_c = c h, c = 2.5 by
 *                                   default (the paper only names a cut-off
 *                                   radius r_c, sec. 2.3)
 *   Shepard term gamma ........... sec. 3.3, Eq. (gamma_disc_renormSPH)
 *   pressure force + boundary .... sec. 3.3, Eq. (sph_pressure_force_disc_weighted)
 *   viscous force ................ sec. 2.3, Eq. (momentum_equation_discretized),
 *                                   Eq. (viscosity_coefficient)
 *   time step per feature ........ sec. 3.5, Eq. (fa_time_step_size)
 *   particle volume, V-bar ....... sec. 3.4.2, Eqs. (particle_volume),
 *                                   (volume_integral)
 *   two-phase control ............ sec. 3.4.2-3.4.4, Eq. (momentum_equation_new)
 *   step order ................... Algorithm 1 (flowchart)
 * Where the paper leaves a point open, the choice made is stated in a
 * comment where it is used.
 *
 * Built with gcc -O2 -ffp-contract=off: no fused multiply-add anywhere, so
 * every expression rounds exactly as written.
 */
#include "sphref.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define MAXF 64
#define MAXH 32

static __thread char g_err[256];
static void set_err(const char *m) { snprintf(g_err, sizeof g_err, "%s", m); }
const char *sphref_last_error(void) { return g_err; }

/* ------------------------------------------------------------------ */
/* features (sec. 3.2)                                                  */
/* ------------------------------------------------------------------ */
enum { T_SI = 0, T_C = 1, T_S = 2, T_V = 3 };
enum { K_VOL, K_BOXSIDE, K_HOLE, K_EDGE3, K_CORNER, K_SHELL, K_LEVEL, K_POLY, K_PCORNER };

typedef struct {
  int type, k, kind;
  int axis, side;           /* BOXSIDE: normal axis and side; EDGE3: direction axis */
  int fax[2], fsd[2];       /* EDGE3: the two fixed axes and their sides */
  int hole;                 /* HOLE: hole index */
  int bits;                 /* CORNER: side bit per axis */
} feat_t;

typedef struct {
  int dim;
  double lo[3], hi[3];
  int nh;
  double hc[MAXH][3], hr[MAXH];
  int ell[MAXH];            /* 1: ellipsoid (unequal semi-axes), 0: ball */
  double ha[MAXH][3];       /* ellipsoid semi-axes */
  double hR[MAXH][9];       /* ellipsoid rotation, row-major: local = R (x - c) */
  int domain;               /* 0 box minus holes, 1 the ball inscribed in the box,
                               2 the positive phase of a gridded level set */
  double dc[3], dR;         /* ball domain: centre and radius */
  const double *phi;        /* level-set domain: node values, counts and box */
  int pn[3];
  double plo[3], phi_hi[3];
  int ncv, ncr;             /* imported curves and corners (level-set domain) */
  int np;                   /* 3D: surface patches the curves split the zero set into */
  const int32_t *coff, *cend, *cpat;
  const double *cpts;
  double cor[MAXF][3];
  int nf;
  feat_t f[MAXF];
} geo_t;

static int geo_build(const sphref_geometry *g, geo_t *G) {
  memset(G, 0, sizeof *G);
  if (!g || (g->dim != 2 && g->dim != 3)) { set_err("dim must be 2 or 3"); return -1; }
  if (g->n_holes < 0 || g->n_holes > MAXH) { set_err("bad hole count"); return -1; }
  G->dim = g->dim;
  for (int a = 0; a < 3; ++a) { G->lo[a] = g->lo[a]; G->hi[a] = g->hi[a]; }
  for (int a = 0; a < g->dim; ++a)
    if (!(g->lo[a] < g->hi[a])) { set_err("empty box"); return -1; }
  if (g->domain < 0 || g->domain > 2) { set_err("domain must be 0, 1 or 2"); return -1; }
  G->domain = g->domain;
  if (G->domain == 2) {
    if (g->n_holes != 0 || !g->phi) { set_err("level-set domain needs phi and no holes"); return -1; }
    G->phi = g->phi;
    for (int a = 0; a < 3; ++a) {
      G->pn[a] = a < g->dim ? g->phi_n[a] : 1;
      G->plo[a] = g->phi_lo[a];
      G->phi_hi[a] = g->phi_hi[a];
      if (a < g->dim && (G->pn[a] < 2 || !(g->phi_hi[a] > g->phi_lo[a]))) {
        set_err("bad level-set grid"); return -1;
      }
    }
    G->f[0] = (feat_t){.type = T_V, .k = g->dim, .kind = K_VOL};
    if (g->n_curves > 0) {
      /* imported curves and corners replace the single zero-set feature; in
       * 3D the curves split the zero set into surface patches */
      int np = g->dim == 3 ? g->n_patches : 0;
      if (!g->curve_off || !g->curve_pts || !g->curve_ends ||
          g->n_corners < 0 || (g->n_corners > 0 && !g->corners) ||
          (g->dim == 2 && g->n_patches != 0) ||
          (g->dim == 3 && (np < 1 || !g->curve_patches)) ||
          1 + np + g->n_curves + g->n_corners > MAXF) {
        set_err("bad imported curves"); return -1;
      }
      G->ncv = g->n_curves;
      G->ncr = g->n_corners;
      G->np = np;
      G->coff = g->curve_off;
      G->cend = g->curve_ends;
      G->cpat = g->curve_patches;
      G->cpts = g->curve_pts;
      for (int c = 0; c < G->ncv; ++c) {
        if (g->curve_off[c + 1] - g->curve_off[c] < 2) { set_err("a curve needs two points"); return -1; }
        for (int k = g->curve_off[c]; k + 1 < g->curve_off[c + 1]; ++k) {
          const double *p0 = g->curve_pts + 3 * k, *p1 = p0 + 3;
          if (p0[0] == p1[0] && p0[1] == p1[1] && (g->dim == 2 || p0[2] == p1[2])) {
            set_err("consecutive curve points must differ"); return -1;
          }
        }
        for (int e = 0; e < 2; ++e) {
          if (g->curve_ends[2 * c + e] < -1 || g->curve_ends[2 * c + e] >= G->ncr) {
            set_err("bad curve end"); return -1;
          }
          if (np > 0 && (g->curve_patches[2 * c + e] < -1 || g->curve_patches[2 * c + e] >= np)) {
            set_err("bad curve patch"); return -1;
          }
        }
      }
      for (int m = 0; m < G->ncr; ++m)
        for (int a = 0; a < 3; ++a) G->cor[m][a] = g->corners[3 * m + a];
      int nf = 1;
      for (int p = 0; p < np; ++p)
        G->f[nf++] = (feat_t){.type = T_S, .k = 2, .kind = K_LEVEL, .hole = p};
      for (int c = 0; c < G->ncv; ++c)
        G->f[nf++] = (feat_t){.type = T_C, .k = 1, .kind = K_POLY, .hole = c};
      for (int m = 0; m < G->ncr; ++m)
        G->f[nf++] = (feat_t){.type = T_SI, .k = 0, .kind = K_PCORNER, .hole = m};
      G->nf = nf;
      return 0;
    }
    G->f[1] = (feat_t){.type = g->dim == 2 ? T_C : T_S, .k = g->dim - 1, .kind = K_LEVEL};
    G->nf = 2;
    return 0;
  }
  if (G->domain == 1) {
    /* the ball (disc) inscribed in a cubic box: features volume and sphere */
    double e0 = g->hi[0] - g->lo[0];
    for (int a = 1; a < g->dim; ++a)
      if (fabs((g->hi[a] - g->lo[a]) - e0) > 1e-12 * e0) { set_err("ball domain needs a cubic box"); return -1; }
    if (g->n_holes != 0) { set_err("ball domain takes no holes"); return -1; }
    for (int a = 0; a < 3; ++a) G->dc[a] = a < g->dim ? 0.5 * (g->lo[a] + g->hi[a]) : 0.0;
    G->dR = 0.5 * e0;
    G->f[0] = (feat_t){.type = T_V, .k = g->dim, .kind = K_VOL};
    G->f[1] = (feat_t){.type = g->dim == 2 ? T_C : T_S, .k = g->dim - 1, .kind = K_SHELL};
    G->nf = 2;
    return 0;
  }
  G->nh = g->n_holes;
  for (int q = 0; q < G->nh; ++q) {
    const double *H = g->holes + 15 * q;
    int D = g->dim;
    for (int a = 0; a < D; ++a)
      if (!(H[3 + a] > 0)) { set_err("hole semi-axes must be positive"); return -1; }
    for (int a = 0; a < 3; ++a) G->hc[q][a] = H[a];
    G->hr[q] = H[3];
    G->ell[q] = D == 2 ? H[4] != H[3] : (H[4] != H[3] || H[5] != H[3]);
    for (int a = 0; a < 3; ++a) G->ha[q][a] = H[3 + a];
    for (int e = 0; e < 9; ++e) G->hR[q][e] = H[6 + e];
    if (G->ell[q]) {               /* the rotation must be orthonormal */
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
          double s = 0.0;
          for (int m = 0; m < 3; ++m) s = s + H[6 + 3 * m + r] * H[6 + 3 * m + c];
          if (fabs(s - (r == c ? 1.0 : 0.0)) > 1e-9) { set_err("hole rotation not orthonormal"); return -1; }
        }
    }
  }
  int D = G->dim, nf = 0;
  G->f[nf++] = (feat_t){.type = T_V, .k = D, .kind = K_VOL};
  for (int a = 0; a < D; ++a)
    for (int s = 0; s < 2; ++s)
      G->f[nf++] = (feat_t){.type = D == 2 ? T_C : T_S, .k = D - 1,
                            .kind = K_BOXSIDE, .axis = a, .side = s};
  for (int q = 0; q < G->nh; ++q)
    G->f[nf++] = (feat_t){.type = D == 2 ? T_C : T_S, .k = D - 1,
                          .kind = K_HOLE, .hole = q};
  if (D == 3) {
    for (int a = 0; a < 3; ++a) {
      int b = a == 0 ? 1 : 0, c = a == 2 ? 1 : 2;
      for (int q = 0; q < 4; ++q) {
        feat_t e = {.type = T_C, .k = 1, .kind = K_EDGE3, .axis = a};
        e.fax[0] = b; e.fsd[0] = q & 1;
        e.fax[1] = c; e.fsd[1] = (q >> 1) & 1;
        G->f[nf++] = e;
      }
    }
  }
  for (int c = 0; c < (1 << D); ++c)
    G->f[nf++] = (feat_t){.type = T_SI, .k = 0, .kind = K_CORNER, .bits = c};
  G->nf = nf;
  return 0;
}

/* fb bounds fi: the lower-dimensional feature fb lies on the boundary of fi
 * (the boundary relation of sec. 3.3 is read as one between adjacent
 * features, since n_b is only defined on i's own boundary; a volume is
 * bounded by every lower-dimensional feature). */
static int bounds(const geo_t *G, int fi, int fb) {
  const feat_t *A = &G->f[fi], *B = &G->f[fb];
  if (B->k >= A->k) return 0;
  switch (A->kind) {
    case K_VOL: return 1;
    case K_BOXSIDE:
      if (B->kind == K_CORNER) return ((B->bits >> A->axis) & 1) == A->side;
      if (B->kind == K_EDGE3)
        return (B->fax[0] == A->axis && B->fsd[0] == A->side) ||
               (B->fax[1] == A->axis && B->fsd[1] == A->side);
      return 0;
    case K_EDGE3:
      if (B->kind == K_CORNER)
        return ((B->bits >> A->fax[0]) & 1) == A->fsd[0] &&
               ((B->bits >> A->fax[1]) & 1) == A->fsd[1];
      return 0;
    case K_POLY:          /* an imported curve is bounded by its end corners */
      return B->kind == K_PCORNER &&
             (G->cend[2 * A->hole] == B->hole || G->cend[2 * A->hole + 1] == B->hole);
    case K_LEVEL:         /* a surface patch: by the curves beside it and their end corners */
      if (G->np == 0) return 0;
      for (int c = 0; c < G->ncv; ++c) {
        if (G->cpat[2 * c] != A->hole && G->cpat[2 * c + 1] != A->hole) continue;
        if (B->kind == K_POLY && B->hole == c) return 1;
        if (B->kind == K_PCORNER && (G->cend[2 * c] == B->hole || G->cend[2 * c + 1] == B->hole)) return 1;
      }
      return 0;
    default: return 0;
  }
}

/* ------------------------------------------------------------------ */
/* ellipsoidal holes: local coordinates y = R (x - c), the hole is       */
/* sum_k (y_k / a_k)^2 <= 1 (sec. 2.1's level set for a quadric)         */
/* ------------------------------------------------------------------ */
static void ell_local(const geo_t *G, int q, const double *x, double *y) {
  int D = G->dim;
  for (int k = 0; k < D; ++k) {
    double s = 0.0;
    for (int m = 0; m < D; ++m) s = s + G->hR[q][3 * k + m] * (x[m] - G->hc[q][m]);
    y[k] = s;
  }
}

static double ell_level(const geo_t *G, int q, const double *y) {
  double s = 0.0;
  for (int k = 0; k < G->dim; ++k) {
    double u = y[k] / G->ha[q][k];
    s = s + u * u;
  }
  return s;
}

/* One Newton step for the closest point: z_k = a_k^2 y_k / (a_k^2 + t) lies
 * on the surface where g(t) = sum_k (a_k y_k / (a_k^2 + t))^2 - 1 = 0, and
 * g'(t) = -2 sum_k (a_k y_k)^2 / (a_k^2 + t)^3. */
static double ell_newton(const geo_t *G, int q, const double *y, double t) {
  double g = -1.0, dg = 0.0;
  for (int k = 0; k < G->dim; ++k) {
    double a = G->ha[q][k];
    double e = a * a + t;
    double u = a * y[k] / e;
    double uu = u * u;
    g = g + uu;
    dg = dg + uu / e;
  }
  return t + g / (2.0 * dg);
}

static void ell_point(const geo_t *G, int q, const double *y, double t, double *z) {
  for (int k = 0; k < G->dim; ++k) {
    double a = G->ha[q][k];
    z[k] = a * a * y[k] / (a * a + t);
  }
}

/* distance from x to the surface of hole q for x outside it (0 inside):
 * g is convex and decreasing for t > -min a^2, so Newton from any point left
 * of the root increases monotonically to it.  g(t) >= |a y|^2 / (max a^2 + t)^2 - 1,
 * so t0 = |a y| - max a^2 (or 0 if negative; g(0) > 0 outside) lies left of
 * the root.  Newton starts there and stops when t no longer increases (at
 * most 64 steps; 11 suffice on [0,1]^3). */
static double ell_dist(const geo_t *G, int q, const double *x) {
  double y[3] = {0, 0, 0}, z[3] = {0, 0, 0};
  ell_local(G, q, x, y);
  if (!(ell_level(G, q, y) > 1.0)) return 0.0;
  double s0 = 0.0, amax2 = 0.0;
  for (int k = 0; k < G->dim; ++k) {
    double a = G->ha[q][k];
    double ay = a * y[k];
    s0 = s0 + ay * ay;
    if (a * a > amax2) amax2 = a * a;
  }
  double t = sqrt(s0) - amax2;
  if (!(t > 0.0)) t = 0.0;
  for (int it = 0; it < 64; ++it) {
    double tn = ell_newton(G, q, y, t);
    if (!(tn > t)) break;
    t = tn;
  }
  ell_point(G, q, y, t, z);
  double s = 0.0;
  for (int k = 0; k < G->dim; ++k) { double d = y[k] - z[k]; s = s + d * d; }
  return sqrt(s);
}

/* closest point on the surface of hole q to a point x near it: eight Newton
 * steps from t = 0 (a fixed count, as the level-set projection of sec. 2.1
 * gives no iteration rule; eight bring offsets up to 3e-3 of the semi-axes
 * to |level - 1| <= 1e-15) */
static void ell_project(const geo_t *G, int q, double *x) {
  int D = G->dim;
  double y[3] = {0, 0, 0}, z[3] = {0, 0, 0};
  ell_local(G, q, x, y);
  double t = 0.0;
  for (int it = 0; it < 8; ++it) t = ell_newton(G, q, y, t);
  ell_point(G, q, y, t, z);
  for (int m = 0; m < D; ++m) {
    double s = 0.0;
    for (int k = 0; k < D; ++k) s = s + G->hR[q][3 * k + m] * z[k];
    x[m] = G->hc[q][m] + s;
  }
}

/* unit normal of hole q's level set at x, pointing out of the hole */
static void ell_normal(const geo_t *G, int q, const double *x, double *n) {
  int D = G->dim;
  double y[3] = {0, 0, 0}, gy[3] = {0, 0, 0};
  ell_local(G, q, x, y);
  for (int k = 0; k < D; ++k) { double a = G->ha[q][k]; gy[k] = y[k] / (a * a); }
  double s = 0.0;
  for (int m = 0; m < D; ++m) {
    double v = 0.0;
    for (int k = 0; k < D; ++k) v = v + G->hR[q][3 * k + m] * gy[k];
    n[m] = v;
    s = s + v * v;
  }
  double r = sqrt(s);
  for (int m = 0; m < D; ++m) n[m] = n[m] / r;
}

static double sg(int side) { return side ? 1.0 : -1.0; }
static double norm3(const double *u) { return sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]); }

/* ------------------------------------------------------------------ */
/* gridded level set (sec. 2.1: phi on a Cartesian background mesh)     */
/* ------------------------------------------------------------------ */
/* phi at x, multilinear in the grid cell of x (coordinates clamped to the
 * grid box as for the gridded sizing), and its gradient: the derivative of
 * that multilinear function inside the cell */
static double ls_phi(const geo_t *G, const double *x, double *grad) {
  int D = G->dim, c[3] = {0, 0, 0};
  double t[3] = {0.0, 0.0, 0.0}, s[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < D; ++a) {
    int n = G->pn[a];
    s[a] = (double)(n - 1) / (G->phi_hi[a] - G->plo[a]);
    double u = (x[a] - G->plo[a]) * s[a];
    if (!(u > 0.0)) u = 0.0;
    if (u > (double)(n - 1)) u = (double)(n - 1);
    double f = floor(u);
    if (f > (double)(n - 2)) f = (double)(n - 2);
    c[a] = (int)f;
    t[a] = u - f;
  }
  int nx = G->pn[0], ny = G->pn[1], nz = D == 3 ? 2 : 1;
  double g[2][2][2], v[2][2], d[2][2];
  for (int dz = 0; dz < nz; ++dz)
    for (int dy = 0; dy < 2; ++dy) {
      int64_t row = ((int64_t)(c[2] + dz) * ny + (c[1] + dy)) * nx + c[0];
      g[dz][dy][0] = G->phi[row];
      g[dz][dy][1] = G->phi[row + 1];
      d[dz][dy] = g[dz][dy][1] - g[dz][dy][0];             /* difference along x */
      v[dz][dy] = g[dz][dy][0] + t[0] * d[dz][dy];          /* lerp along x */
    }
  double w[2], e[2], q[2];
  for (int dz = 0; dz < nz; ++dz) {
    q[dz] = v[dz][1] - v[dz][0];                            /* difference along y */
    w[dz] = v[dz][0] + t[1] * q[dz];                        /* lerp along y */
    e[dz] = d[dz][0] + t[1] * (d[dz][1] - d[dz][0]);        /* x-difference lerped along y */
  }
  grad[0] = grad[1] = grad[2] = 0.0;
  if (D == 2) {
    grad[0] = s[0] * e[0];
    grad[1] = s[1] * q[0];
    return w[0];
  }
  grad[0] = s[0] * (e[0] + t[2] * (e[1] - e[0]));
  grad[1] = s[1] * (q[0] + t[2] * (q[1] - q[0]));
  grad[2] = s[2] * (w[1] - w[0]);
  return w[0] + t[2] * (w[1] - w[0]);
}

/* imported curve c (a polyline; in 2D with the domain on its left): the
 * segment whose closest point to x is nearest (the first one on ties), and
 * that point */
static int poly_closest(const geo_t *G, int c, const double *x, double *q) {
  int D = G->dim;
  int best = G->coff[c];                     /* also when no distance compares */
  for (int a = 0; a < 3; ++a) q[a] = a < D ? G->cpts[3 * best + a] : 0.0;
  double bd = INFINITY;
  for (int k = G->coff[c]; k + 1 < G->coff[c + 1]; ++k) {
    const double *p0 = G->cpts + 3 * k, *p1 = G->cpts + 3 * (k + 1);
    double e[3] = {0, 0, 0}, ee = 0.0, xe = 0.0;
    for (int a = 0; a < D; ++a) {
      e[a] = p1[a] - p0[a];
      ee = ee + e[a] * e[a];
      xe = xe + (x[a] - p0[a]) * e[a];
    }
    double t = ee > 0.0 ? xe / ee : 0.0;
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
    double cp[3] = {0, 0, 0}, d = 0.0;
    for (int a = 0; a < D; ++a) {
      cp[a] = p0[a] + t * e[a];
      d = d + (x[a] - cp[a]) * (x[a] - cp[a]);
    }
    if (d < bd) { bd = d; best = k; for (int a = 0; a < 3; ++a) q[a] = cp[a]; }
  }
  return best;
}

/* unit tangent of segment k of the imported curves (along the curve) */
static void seg_tangent(const geo_t *G, int k, double *t) {
  const double *p0 = G->cpts + 3 * k, *p1 = G->cpts + 3 * (k + 1);
  double e[3] = {0, 0, 0}, s = 0.0;
  for (int a = 0; a < G->dim; ++a) { e[a] = p1[a] - p0[a]; s = s + e[a] * e[a]; }
  double l = sqrt(s);
  for (int a = 0; a < 3; ++a) t[a] = e[a] / l;
}

/* unit normal of the level set at x, pointing to increasing phi (into the
 * domain); 0 where the gradient vanishes */
static void ls_unit(const geo_t *G, const double *x, double *m) {
  double gr[3];
  ls_phi(G, x, gr);
  double s = 0.0;
  for (int a = 0; a < G->dim; ++a) s = s + gr[a] * gr[a];
  double r = sqrt(s);
  m[0] = m[1] = m[2] = 0.0;
  if (!(r > 0.0)) return;
  for (int a = 0; a < G->dim; ++a) m[a] = gr[a] / r;
}

/* closest point on the zero level set, read as a fixed count of Newton
 * steps along the gradient, x <- x - phi grad / |grad|^2 (sec. 2.1 gives
 * no iteration rule) */
static void ls_project(const geo_t *G, double *x) {
  int D = G->dim;
  for (int it = 0; it < 12; ++it) {
    double gr[3];
    double p = ls_phi(G, x, gr);
    double gg = 0.0;
    for (int a = 0; a < D; ++a) gg = gg + gr[a] * gr[a];
    if (!(gg > 0.0)) return;
    for (int a = 0; a < D; ++a) x[a] = x[a] - p * gr[a] / gg;
  }
}

/* outward normal n_b of feature fi's boundary at boundary particle b
 * (sec. 3.3, Eq. (gradient_operator_renormSPH_bypart): n points out of the
 * domain of i; at box edges and corners the normalised sum of the adjacent
 * face normals, within a face the in-face conormal, on a curve the outward
 * tangent). */
static void bnormal(const geo_t *G, int fi, int fb, const double *xb, const double *xi, double *n) {
  const feat_t *A = &G->f[fi], *B = &G->f[fb];
  int D = G->dim;
  n[0] = n[1] = n[2] = 0.0;
  if (A->kind == K_VOL) {
    if (B->kind == K_BOXSIDE) {
      n[B->axis] = sg(B->side);
    } else if (B->kind == K_HOLE && G->ell[B->hole]) {
      /* out of the domain = into the hole, against its level set's normal */
      ell_normal(G, B->hole, xb, n);
      for (int a = 0; a < D; ++a) n[a] = -n[a];
    } else if (B->kind == K_HOLE) {
      /* out of the domain = into the hole, towards its centre */
      double d[3] = {0, 0, 0}, s = 0.0;
      for (int a = 0; a < D; ++a) { d[a] = G->hc[B->hole][a] - xb[a]; s = s + d[a] * d[a]; }
      double r = sqrt(s);
      for (int a = 0; a < D; ++a) n[a] = d[a] / r;
    } else if (B->kind == K_POLY && D == 3) {
      /* a 3D curve on the zero set: towards decreasing phi, as on a patch */
      ls_unit(G, xb, n);
      for (int a = 0; a < 3; ++a) n[a] = -n[a];
    } else if (B->kind == K_PCORNER && D == 3) {
      /* a 3D corner: towards decreasing phi at the corner point */
      ls_unit(G, G->cor[B->hole], n);
      for (int a = 0; a < 3; ++a) n[a] = -n[a];
    } else if (B->kind == K_POLY) {
      /* out of the domain = the right of the curve's closest segment */
      double q[3], t[3];
      seg_tangent(G, poly_closest(G, B->hole, xb, q), t);
      n[0] = t[1]; n[1] = -t[0];
    } else if (B->kind == K_PCORNER) {
      /* the normalised sum of the outward normals of the end segments of
       * the curves that meet at the corner */
      double s0 = 0.0, s1 = 0.0;
      for (int c = 0; c < G->ncv; ++c)
        for (int e = 0; e < 2; ++e) {
          if (G->cend[2 * c + e] != B->hole) continue;
          int k = e == 0 ? G->coff[c] : G->coff[c + 1] - 2;
          double t[3];
          seg_tangent(G, k, t);
          s0 = s0 + t[1]; s1 = s1 - t[0];
        }
      double l = sqrt(s0 * s0 + s1 * s1);
      if (l > 0.0) { n[0] = s0 / l; n[1] = s1 / l; }
    } else if (B->kind == K_LEVEL) {
      /* out of the domain = towards decreasing phi */
      ls_unit(G, xb, n);
      for (int a = 0; a < D; ++a) n[a] = -n[a];
    } else if (B->kind == K_SHELL) {
      /* out of the ball domain: radially outwards */
      double d[3] = {0, 0, 0}, s = 0.0;
      for (int a = 0; a < D; ++a) { d[a] = xb[a] - G->dc[a]; s = s + d[a] * d[a]; }
      double r = sqrt(s);
      for (int a = 0; a < D; ++a) n[a] = d[a] / r;
    } else if (B->kind == K_EDGE3) {
      double inv = 1.0 / sqrt(2.0);
      n[B->fax[0]] = sg(B->fsd[0]) * inv;
      n[B->fax[1]] = sg(B->fsd[1]) * inv;
    } else if (B->kind == K_CORNER) {
      double inv = 1.0 / sqrt((double)D);
      for (int a = 0; a < D; ++a) n[a] = sg((B->bits >> a) & 1) * inv;
    }
  } else if (A->kind == K_BOXSIDE && D == 3) {
    if (B->kind == K_EDGE3) {
      int o = B->fax[0] == A->axis ? 1 : 0;   /* the fixed axis that is not the face normal */
      n[B->fax[o]] = sg(B->fsd[o]);
    } else if (B->kind == K_CORNER) {
      double inv = 1.0 / sqrt(2.0);
      for (int a = 0; a < 3; ++a)
        if (a != A->axis) n[a] = sg((B->bits >> a) & 1) * inv;
    }
  } else if (A->kind == K_BOXSIDE && D == 2) {
    int o = 1 - A->axis;                      /* the edge runs along axis o */
    n[o] = sg((B->bits >> o) & 1);
  } else if (A->kind == K_EDGE3) {
    n[A->axis] = sg((B->bits >> A->axis) & 1);
  } else if (A->kind == K_POLY) {
    /* out of the curve at its end corner: along the end segment, away from
     * the curve's interior */
    int c = A->hole;
    double t[3];
    if (G->cend[2 * c] == B->hole) {
      seg_tangent(G, G->coff[c], t);
      for (int a = 0; a < 3; ++a) n[a] = -t[a];
    } else {
      seg_tangent(G, G->coff[c + 1] - 2, t);
      for (int a = 0; a < 3; ++a) n[a] = t[a];
    }
  } else if (A->kind == K_LEVEL) {
    /* a 3D surface patch at a curve or corner beside it: the direction from
     * the particle i to b within i's tangent plane (the patch normal m at x_i
     * removed), and at a curve also without the part along the curve's
     * tangent t at b (its closest segment), normalised:
     *   n = (I - t t^T)(I - m m^T)(x_b - x_i) / |.|
     * For a flat patch and a straight curve this is the patch's outward
     * conormal, as the in-face normal at a box edge. */
    double m[3], d[3], dm = 0.0;
    ls_unit(G, xi, m);
    for (int a = 0; a < 3; ++a) { d[a] = xb[a] - xi[a]; dm = dm + d[a] * m[a]; }
    for (int a = 0; a < 3; ++a) d[a] = d[a] - dm * m[a];
    if (B->kind == K_POLY) {
      double q[3], t[3], dt = 0.0;
      seg_tangent(G, poly_closest(G, B->hole, xb, q), t);
      for (int a = 0; a < 3; ++a) dt = dt + d[a] * t[a];
      for (int a = 0; a < 3; ++a) d[a] = d[a] - dt * t[a];
    }
    double l = norm3(d);
    if (l > 0.0)
      for (int a = 0; a < 3; ++a) n[a] = d[a] / l;
  }
}

/* tangent projection T_i u of sec. 3.6's "map onto feature k" (its cited
 * equations are not available; read as):
 * identity for volume particles, remove the normal part on surfaces, keep the
 * tangent part on curves, zero for singular particles. */
static void tproject(const geo_t *G, int fi, const double *x, double *u) {
  const feat_t *A = &G->f[fi];
  int D = G->dim;
  switch (A->kind) {
    case K_VOL: return;
    case K_BOXSIDE: u[A->axis] = 0.0; return;
    case K_EDGE3: {
      double keep = u[A->axis];
      u[0] = u[1] = u[2] = 0.0;
      u[A->axis] = keep;
      return;
    }
    case K_HOLE: {
      const double *c = G->hc[A->hole];
      if (G->ell[A->hole]) {
        double m[3] = {0, 0, 0};
        ell_normal(G, A->hole, x, m);
        if (D == 2) {                     /* keep the part along the tangent (-n1, n0) */
          double ut = u[0] * (-m[1]) + u[1] * m[0];
          u[0] = ut * (-m[1]); u[1] = ut * m[0];
        } else {                          /* remove the normal part */
          double un = u[0] * m[0] + u[1] * m[1] + u[2] * m[2];
          for (int a = 0; a < 3; ++a) u[a] = u[a] - un * m[a];
        }
        return;
      }
      if (D == 2) {
        double t0 = -(x[1] - c[1]), t1 = x[0] - c[0];
        double tl = sqrt(t0 * t0 + t1 * t1);
        t0 = t0 / tl; t1 = t1 / tl;
        double ut = u[0] * t0 + u[1] * t1;
        u[0] = ut * t0; u[1] = ut * t1;
      } else {
        double m[3], s = 0.0;
        for (int a = 0; a < 3; ++a) { m[a] = x[a] - c[a]; s = s + m[a] * m[a]; }
        double r = sqrt(s);
        for (int a = 0; a < 3; ++a) m[a] = m[a] / r;
        double un = u[0] * m[0] + u[1] * m[1] + u[2] * m[2];
        for (int a = 0; a < 3; ++a) u[a] = u[a] - un * m[a];
      }
      return;
    }
    case K_POLY: {                        /* keep the part along the closest segment */
      double q[3], t[3];
      seg_tangent(G, poly_closest(G, A->hole, x, q), t);
      if (D == 2) {
        double ut = u[0] * t[0] + u[1] * t[1];
        u[0] = ut * t[0]; u[1] = ut * t[1]; u[2] = 0.0;
      } else {
        double ut = u[0] * t[0] + u[1] * t[1] + u[2] * t[2];
        for (int a = 0; a < 3; ++a) u[a] = ut * t[a];
      }
      return;
    }
    case K_LEVEL: {
      double m[3];
      ls_unit(G, x, m);
      if (D == 2) {                       /* keep the part along the tangent (-m1, m0) */
        double ut = u[0] * (-m[1]) + u[1] * m[0];
        u[0] = ut * (-m[1]); u[1] = ut * m[0];
      } else {                            /* remove the normal part */
        double un = u[0] * m[0] + u[1] * m[1] + u[2] * m[2];
        for (int a = 0; a < 3; ++a) u[a] = u[a] - un * m[a];
      }
      return;
    }
    case K_SHELL: {
      const double *c = G->dc;
      if (D == 2) {                       /* keep the part along the circle's tangent */
        double t0 = -(x[1] - c[1]), t1 = x[0] - c[0];
        double tl = sqrt(t0 * t0 + t1 * t1);
        t0 = t0 / tl; t1 = t1 / tl;
        double ut = u[0] * t0 + u[1] * t1;
        u[0] = ut * t0; u[1] = ut * t1;
      } else {                            /* remove the radial part */
        double m[3], s = 0.0;
        for (int a = 0; a < 3; ++a) { m[a] = x[a] - c[a]; s = s + m[a] * m[a]; }
        double r = sqrt(s);
        for (int a = 0; a < 3; ++a) m[a] = m[a] / r;
        double un = u[0] * m[0] + u[1] * m[1] + u[2] * m[2];
        for (int a = 0; a < 3; ++a) u[a] = u[a] - un * m[a];
      }
      return;
    }
    default: u[0] = u[1] = u[2] = 0.0; return;
  }
}

static double clampd(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* closest-point projection of x onto feature fi (sec. 3.6's mapping, read
 * as the closest point: clamped to a face or edge segment, radial on circles
 * and spheres, Newton on ellipses and ellipsoids) */
static void pproject(const geo_t *G, int fi, double *x) {
  const feat_t *A = &G->f[fi];
  int D = G->dim;
  switch (A->kind) {
    case K_BOXSIDE:
      for (int a = 0; a < D; ++a) x[a] = clampd(x[a], G->lo[a], G->hi[a]);
      x[A->axis] = A->side ? G->hi[A->axis] : G->lo[A->axis];
      return;
    case K_EDGE3:
      x[A->axis] = clampd(x[A->axis], G->lo[A->axis], G->hi[A->axis]);
      for (int q = 0; q < 2; ++q)
        x[A->fax[q]] = A->fsd[q] ? G->hi[A->fax[q]] : G->lo[A->fax[q]];
      return;
    case K_HOLE: {
      if (G->ell[A->hole]) { ell_project(G, A->hole, x); return; }
      const double *c = G->hc[A->hole];
      double d[3] = {0, 0, 0}, s = 0.0;
      for (int a = 0; a < D; ++a) { d[a] = x[a] - c[a]; s = s + d[a] * d[a]; }
      double r = sqrt(s);
      for (int a = 0; a < D; ++a) x[a] = c[a] + G->hr[A->hole] * (d[a] / r);
      return;
    }
    case K_CORNER:
      for (int a = 0; a < D; ++a) x[a] = ((A->bits >> a) & 1) ? G->hi[a] : G->lo[a];
      return;
    case K_LEVEL: ls_project(G, x); return;
    case K_POLY: {
      double q[3];
      poly_closest(G, A->hole, x, q);
      for (int a = 0; a < D; ++a) x[a] = q[a];
      return;
    }
    case K_PCORNER:
      for (int a = 0; a < 3; ++a) x[a] = G->cor[A->hole][a];
      return;
    case K_SHELL: {
      double d[3] = {0, 0, 0}, s = 0.0;
      for (int a = 0; a < D; ++a) { d[a] = x[a] - G->dc[a]; s = s + d[a] * d[a]; }
      double r = sqrt(s);
      for (int a = 0; a < D; ++a) x[a] = G->dc[a] + G->dR * (d[a] / r);
      return;
    }
    default: return;
  }
}

/* phi(x) > 0: strictly inside the box and strictly outside every hole, or
 * strictly inside the ball domain (sec. 2.1) */
static int inside(const geo_t *G, const double *x) {
  int D = G->dim;
  if (G->domain == 1) {
    double s = 0.0;
    for (int a = 0; a < D; ++a) { double d = x[a] - G->dc[a]; s = s + d * d; }
    return s < G->dR * G->dR;
  }
  if (G->domain == 2) {
    for (int a = 0; a < D; ++a)
      if (!(x[a] > G->lo[a] && x[a] < G->hi[a])) return 0;
    double gr[3];
    return ls_phi(G, x, gr) > 0.0;
  }
  for (int a = 0; a < D; ++a)
    if (!(x[a] > G->lo[a] && x[a] < G->hi[a])) return 0;
  for (int q = 0; q < G->nh; ++q) {
    if (G->ell[q]) {
      double y[3] = {0, 0, 0};
      ell_local(G, q, x, y);
      if (!(ell_level(G, q, y) > 1.0)) return 0;
      continue;
    }
    double s = 0.0;
    for (int a = 0; a < D; ++a) { double d = x[a] - G->hc[q][a]; s = s + d * d; }
    double r = G->hr[q];
    if (!(s > r * r)) return 0;
  }
  return 1;
}

/* ------------------------------------------------------------------ */
/* target feature size h_t(x) (sec. 2.2; h_i = h_t(x_i) each step)       */
/* ------------------------------------------------------------------ */

/* h sampled on a Cartesian background grid (sec. 2.2 computes h_t on the
 * background mesh), interpolated multilinearly: along x between the nodes
 * of the cell, then along y between those results, then along z */
static double grid_h(const sphref_sizing *S, int D, const double *x) {
  int c[3] = {0, 0, 0};
  double t[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < D; ++a) {
    int n = S->grid_n[a];
    double s = (double)(n - 1) / (S->grid_hi[a] - S->grid_lo[a]);
    double u = (x[a] - S->grid_lo[a]) * s;
    if (!(u > 0.0)) u = 0.0;                 /* also a NaN */
    if (u > (double)(n - 1)) u = (double)(n - 1);
    double f = floor(u);
    if (f > (double)(n - 2)) f = (double)(n - 2);
    c[a] = (int)f;
    t[a] = u - f;
  }
  int nx = S->grid_n[0], ny = S->grid_n[1];
  double v[2][2];                            /* [z corner][y corner], lerped along x */
  for (int dz = 0; dz < (D == 3 ? 2 : 1); ++dz)
    for (int dy = 0; dy < 2; ++dy) {
      int64_t row = ((int64_t)(c[2] + dz) * ny + (c[1] + dy)) * nx + c[0];
      double g0 = S->grid[row], g1 = S->grid[row + 1];
      v[dz][dy] = g0 + t[0] * (g1 - g0);
    }
  double w0 = v[0][0] + t[1] * (v[0][1] - v[0][0]);
  if (D == 2) return w0;
  double w1 = v[1][0] + t[1] * (v[1][1] - v[1][0]);
  return w0 + t[2] * (w1 - w0);
}

/* a bound of |grad h| for the gridded sizing: the multilinear interpolant's
 * derivative along axis a is a weighted mean of node differences along a */
static double grid_lipschitz(const sphref_sizing *S, int D) {
  double sum = 0.0;
  int n[3] = {S->grid_n[0], S->grid_n[1], D == 3 ? S->grid_n[2] : 1};
  for (int a = 0; a < D; ++a) {
    double m = 0.0;
    int st = a == 0 ? 1 : (a == 1 ? n[0] : n[0] * n[1]);
    for (int k = 0; k < n[2]; ++k)
      for (int j = 0; j < n[1]; ++j)
        for (int i = 0; i < n[0]; ++i) {
          int id[3] = {i, j, k};
          if (id[a] + 1 >= n[a]) continue;
          int64_t p = ((int64_t)k * n[1] + j) * n[0] + i;
          double d = fabs(S->grid[p + st] - S->grid[p]);
          if (d > m) m = d;
        }
    double g = m * (double)(n[a] - 1) / (S->grid_hi[a] - S->grid_lo[a]);
    sum = sum + g * g;
  }
  return sqrt(sum);
}
static double h_at(const geo_t *G, const sphref_sizing *S, const double *x) {
  int D = G->dim;
  if (S->kind == 0) return S->h0;
  if (S->kind == 1) {
    double s = 0.0;
    for (int a = 0; a < D; ++a) { double d = x[a] - S->point[a]; s = s + d * d; }
    return S->h0 + S->grad * sqrt(s);
  }
  if (S->kind == 4) return grid_h(S, D, x);
  if (S->kind == 3) {     /* graded both ways from the sphere |x - point| = dcap */
    double s = 0.0;
    for (int a = 0; a < D; ++a) { double d = x[a] - S->point[a]; s = s + d * d; }
    return S->h0 + S->grad * fabs(sqrt(s) - S->dcap);
  }
  double dmin = INFINITY;
  for (int q = 0; q < G->nh; ++q) {
    double d;
    if (G->ell[q]) {
      d = ell_dist(G, q, x);
    } else {
      double s = 0.0;
      for (int a = 0; a < D; ++a) { double e = x[a] - G->hc[q][a]; s = s + e * e; }
      d = fabs(sqrt(s) - G->hr[q]);
    }
    if (d < dmin) dmin = d;
  }
  if (S->dcap < dmin) dmin = S->dcap;
  return S->h0 * (1.0 + S->grad * dmin);
}

/* ------------------------------------------------------------------ */
/* kernel: Wendland C2 (sec. 2.3 names only a cut-off radius), reaching  */
/* two smoothing lengths, in the intrinsic dimension k of the feature     */
/* ------------------------------------------------------------------ */
static double kalpha(int k) {
  if (k == 1) return 5.0 / 8.0;
  if (k == 2) return 7.0 / (4.0 * M_PI);
  return 21.0 / (16.0 * M_PI);
}
static double hpow(double h, int k) {
  double p = 1.0;
  for (int e = 0; e < k; ++e) p = p * h;
  return p;
}
double sphref_W(int32_t k, double r, double h) {
  double q = r / h;
  if (!(q < 2.0)) return 0.0;
  double t = 1.0 - 0.5 * q;
  double w = k == 1 ? t * t * t * (1.0 + 1.5 * q) : t * t * t * t * (1.0 + 2.0 * q);
  return kalpha(k) * w / hpow(h, k);
}
double sphref_dWdr(int32_t k, double r, double h) {
  double q = r / h;
  if (!(q < 2.0)) return 0.0;
  double t = 1.0 - 0.5 * q;
  double dw = k == 1 ? -3.0 * q * t * t : -5.0 * q * t * t * t;
  return kalpha(k) * dw / hpow(h, k + 1);
}
/* (dW/dr)/r, the same quantity written so that it stays finite at r = 0:
 * with q = r/h, (dW/dr)/r = alpha * (w'(q)/q) / h^(k+2). */
static double dWdr_over_r(int k, double r, double h) {
  double q = r / h;
  if (!(q < 2.0)) return 0.0;
  double t = 1.0 - 0.5 * q;
  double dwq = k == 1 ? -3.0 * t * t : -5.0 * t * t * t;
  return kalpha(k) * dwq / hpow(h, k + 2);
}

/* ------------------------------------------------------------------ */
/* job                                                                  */
/* ------------------------------------------------------------------ */
enum { PH_ONE = 1, PH_RAMP = 2, PH_TWO = 3, PH_FROZEN = 4 };

typedef struct {
  int phase, n_ph, reset_next, nring, nwin, count;
  double dt_prev, dt1, dt, esys, vbar, a_last, a_prev;
  double ring[64];
} grp_t;

struct sphref_job {
  geo_t G;
  sphref_sizing S;
  sphref_params P;
  int64_t n;
  double *x, *v, *h, *ap, *a, *vt, *Vt, *gam, *eta;
  int32_t *f;
  grp_t g[MAXF];
  /* neighbour lists of the current step */
  int64_t *off;
  int32_t *nb;
  int8_t *rel;
  int64_t cap;
  /* counters */
  int64_t steps, escaped, inter_total, inter_last;
  int state_error;
};

static int ftype(const sphref_job *J, int64_t i) { return J->G.f[J->f[i]].type; }

int32_t sphref_n_features(const sphref_geometry *g) {
  geo_t G;
  if (geo_build(g, &G)) return -1;
  return G.nf;
}
int32_t sphref_feature_type(const sphref_geometry *g, int32_t f) {
  geo_t G;
  if (geo_build(g, &G) || f < 0 || f >= G.nf) return -1;
  return G.f[f].type;
}
double sphref_h_at(const sphref_geometry *g, const sphref_sizing *s, const double *x) {
  geo_t G;
  if (geo_build(g, &G)) return NAN;
  return h_at(&G, s, x);
}
int32_t sphref_project(const sphref_geometry *g, int32_t f, double *x) {
  geo_t G;
  if (geo_build(g, &G) || f < 0 || f >= G.nf) return -1;
  pproject(&G, f, x);
  return 0;
}
int32_t sphref_boundary_normal_at(const sphref_geometry *g, int32_t fi, int32_t fb,
                                  const double *xb, const double *xi, double *n) {
  geo_t G;
  if (geo_build(g, &G) || fi < 0 || fb < 0 || fi >= G.nf || fb >= G.nf) return -1;
  if (!bounds(&G, fi, fb)) { n[0] = n[1] = n[2] = 0.0; return 0; }
  if (G.f[fi].kind == K_LEVEL && !xi) { set_err("this normal depends on x_i"); return -1; }
  bnormal(&G, fi, fb, xb, xi, n);
  return 1;
}
int32_t sphref_boundary_normal(const sphref_geometry *g, int32_t fi, int32_t fb,
                               const double *xb, double *n) {
  return sphref_boundary_normal_at(g, fi, fb, xb, NULL, n);
}

static void grp_init(grp_t *g) {
  memset(g, 0, sizeof *g);
  g->phase = PH_ONE;
  g->esys = INFINITY;
}

int32_t sphref_create(const sphref_geometry *g, const sphref_sizing *s,
                      const sphref_params *p, int64_t n, const double *xyz,
                      const int32_t *feature, sphref_job **out) {
  if (!out || !s || !p || n < 0 || (n > 0 && (!xyz || !feature))) { set_err("bad argument"); return -1; }
  *out = NULL;
  sphref_job *J = calloc(1, sizeof *J);
  if (!J) { set_err("out of memory"); return -1; }
  if (geo_build(g, &J->G)) { free(J); return -1; }
  if (p->window_samples < 1 || p->window_samples > 64 || p->sample_every < 1 ||
      p->reset_period < 1 || p->ramp_halving < 1) {
    set_err("bad control parameters");
    free(J);
    return -1;
  }
  J->S = *s;
  J->P = *p;
  J->n = n;
  size_t n3 = (size_t)(n > 0 ? n : 1) * 3;
  J->x = calloc(n3, sizeof(double));
  J->v = calloc(n3, sizeof(double));
  J->ap = calloc(n3, sizeof(double));
  J->a = calloc(n3, sizeof(double));
  J->vt = calloc(n3, sizeof(double));
  J->h = calloc(n3 / 3, sizeof(double));
  J->Vt = calloc(n3 / 3, sizeof(double));
  J->gam = calloc(n3 / 3, sizeof(double));
  J->eta = calloc(n3 / 3, sizeof(double));
  J->f = calloc(n3 / 3, sizeof(int32_t));
  J->off = calloc(n3 / 3 + 1, sizeof(int64_t));
  if (!J->x || !J->v || !J->ap || !J->a || !J->vt || !J->h || !J->Vt || !J->gam ||
      !J->eta || !J->f || !J->off) {
    set_err("out of memory");
    sphref_destroy(J);
    return -1;
  }
  for (int64_t i = 0; i < n; ++i) {
    if (feature[i] < 0 || feature[i] >= J->G.nf) { set_err("feature index out of range"); sphref_destroy(J); return -1; }
    J->f[i] = feature[i];
    for (int a = 0; a < 3; ++a) J->x[3 * i + a] = a < J->G.dim ? xyz[3 * i + a] : 0.0;
  }
  for (int q = 0; q < J->G.nf; ++q) grp_init(&J->g[q]);
  for (int64_t i = 0; i < n; ++i) J->g[J->f[i]].count++;
  *out = J;
  return 0;
}

void sphref_destroy(sphref_job *J) {
  if (!J) return;
  free(J->x); free(J->v); free(J->h); free(J->ap); free(J->a); free(J->vt);
  free(J->Vt); free(J->gam); free(J->eta); free(J->f); free(J->off); free(J->nb); free(J->rel);
  free(J);
}

int32_t sphref_set_state(sphref_job *J, const double *xyz, const double *vel) {
  for (int64_t i = 0; i < J->n; ++i)
    for (int a = 0; a < 3; ++a) {
      if (xyz) J->x[3 * i + a] = a < J->G.dim ? xyz[3 * i + a] : 0.0;
      if (vel) J->v[3 * i + a] = a < J->G.dim ? vel[3 * i + a] : 0.0;
    }
  return 0;
}

int32_t sphref_get_state(sphref_job *J, double *xyz, double *vel) {
  if (xyz) memcpy(xyz, J->x, sizeof(double) * 3 * (size_t)J->n);
  if (vel) memcpy(vel, J->v, sizeof(double) * 3 * (size_t)J->n);
  return 0;
}

int32_t sphref_get_field(sphref_job *J, int32_t which, double *out) {
  size_t n = (size_t)J->n;
  switch (which) {
    case SPHREF_F_H: memcpy(out, J->h, sizeof(double) * n); return 0;
    case SPHREF_F_AP: memcpy(out, J->ap, sizeof(double) * 3 * n); return 0;
    case SPHREF_F_A: memcpy(out, J->a, sizeof(double) * 3 * n); return 0;
    case SPHREF_F_VT: memcpy(out, J->Vt, sizeof(double) * n); return 0;
    case SPHREF_F_GAMMA: memcpy(out, J->gam, sizeof(double) * n); return 0;
    case SPHREF_F_VMID: memcpy(out, J->vt, sizeof(double) * 3 * n); return 0;
    default: set_err("unknown field"); return -1;
  }
}

/* ------------------------------------------------------------------ */
/* neighbour lists (Algorithm 1: "construct Verlet neighbor list")       */
/* ------------------------------------------------------------------ */
/* relation of j to i (sec. 3.3 interaction hierarchy, boundary relation
 * between adjacent features as in bounds()):
 * 1 same type and index, 2 j bounds i's feature, 0 no interaction. */
static int relation(const sphref_job *J, int64_t i, int64_t j) {
  if (J->f[i] == J->f[j]) return 1;
  return bounds(&J->G, J->f[i], J->f[j]) ? 2 : 0;
}

/* cut-off radius r_c in units of h (sec. 2.3 gives no value; 2 by
 * default, the Wendland kernel's own support of two smoothing lengths at
 * smoothing length h), and the kernel's smoothing length per unit h (the
 * kernel reaches 2 smoothing lengths) */
static double rc_ratio(const sphref_params *P) {
  return P->kernel_support > 0.0 ? P->kernel_support : 2.0;
}
static double klen(const sphref_params *P) { return 0.5 * rc_ratio(P); }

/* factor on the boundary term.  Eq. (sph_pressure_force_disc_weighted)
 * carries none: with factor 1 (the default) and weight 1/h_b the boundary
 * sum is the surface integral of Eq. (gradient_operator_renormSPH_bypart),
 * which for evenly spaced particles cancels the truncated interior sum.  A
 * factor above 1 is a calibration, not a reading: factor 2 moves the first
 * particle off a boundary from half a spacing to one spacing. */
static double bscale(const sphref_params *P) {
  return P->boundary_scale > 0.0 ? P->boundary_scale : 1.0;
}

/* the pair predicate (symmetric, and covering both kernel supports used,
 * W(., h_i) and W(., h_ij)): |x_i - x_j|^2 < c^2 max(h_i,h_j)^2 with
 * c = r_c / h, the squared distance summed over axes in order, no fused
 * operations */
static int within(const sphref_job *J, int64_t i, int64_t j) {
  int D = J->G.dim;
  double s = 0.0;
  for (int a = 0; a < D; ++a) {
    double d = J->x[3 * i + a] - J->x[3 * j + a];
    s = s + d * d;
  }
  double m = J->h[i] > J->h[j] ? J->h[i] : J->h[j];
  double c = rc_ratio(&J->P);
  return s < (c * c) * (m * m);
}

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}
static int cmp_i32_desc(const void *a, const void *b) { return cmp_i32(b, a); }

/* candidates of particle i from the bucket grid that pass the predicate and
 * have a relation; writes their ids to out (if not NULL) and returns how
 * many there are */
typedef struct {
  int64_t nc[3];
  const int64_t *cstart, *cell, *bucket;
} buckets_t;

static int64_t scan_particle(const sphref_job *J, const buckets_t *B, int64_t i, int32_t *out) {
  int D = J->G.dim;
  int64_t ci[3] = {0, 0, 0};
  int64_t c = B->cell[i];
  for (int a = 0; a < D; ++a) { ci[a] = c % B->nc[a]; c /= B->nc[a]; }
  int64_t m = 0;
  for (int64_t dz = (D == 3 ? -1 : 0); dz <= (D == 3 ? 1 : 0); ++dz)
    for (int64_t dy = -1; dy <= 1; ++dy)
      for (int64_t dx = -1; dx <= 1; ++dx) {
        int64_t q[3] = {ci[0] + dx, ci[1] + dy, ci[2] + dz};
        int ok = 1;
        for (int a = 0; a < D; ++a) if (q[a] < 0 || q[a] >= B->nc[a]) ok = 0;
        if (!ok) continue;
        int64_t cc = 0;
        for (int a = D - 1; a >= 0; --a) cc = cc * B->nc[a] + q[a];
        for (int64_t t = B->cstart[cc]; t < B->cstart[cc + 1]; ++t) {
          int64_t j = B->bucket[t];
          if (j == i || !within(J, i, j)) continue;
          if (!relation(J, i, j)) continue;
          if (out) out[m] = (int32_t)j;
          m++;
        }
      }
  return m;
}

/* Lists for every non-singular particle.  A uniform bucket grid of side
 * c max(h) only limits which pairs are tested; the set is exactly the pairs
 * that pass the predicate and have a relation.  Ids are sorted ascending.
 * Each particle's list depends on nothing but the positions and h, so the
 * count and fill passes may run over particles in any order (in parallel in
 * the OpenMP build). */
static int build_lists(sphref_job *J) {
  int D = J->G.dim;
  int64_t n = J->n;
  double hmax = 0.0, lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  for (int64_t i = 0; i < n; ++i) if (J->h[i] > hmax) hmax = J->h[i];
  for (int a = 0; a < D; ++a) { lo[a] = INFINITY; hi[a] = -INFINITY; }
  for (int64_t i = 0; i < n; ++i)
    for (int a = 0; a < D; ++a) {
      double c = J->x[3 * i + a];
      if (!isfinite(c)) { set_err("non-finite position"); return -1; }
      if (c < lo[a]) lo[a] = c;
      if (c > hi[a]) hi[a] = c;
    }
  double cs = rc_ratio(&J->P) * hmax;
  if (!(cs > 0)) cs = 1.0;
  int64_t nc[3] = {1, 1, 1}, ncell = 1;
  for (int a = 0; a < D; ++a) {
    nc[a] = (int64_t)floor((hi[a] - lo[a]) / cs) + 1;
    ncell *= nc[a];
  }
  int64_t *cstart = calloc((size_t)ncell + 1, sizeof(int64_t));
  int64_t *cell = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t *bucket = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t *fill = calloc((size_t)ncell, sizeof(int64_t));
  if (!cstart || !cell || !bucket || !fill) {
    free(cstart); free(cell); free(bucket); free(fill);
    set_err("out of memory");
    return -1;
  }
  for (int64_t i = 0; i < n; ++i) {
    int64_t c = 0;
    for (int a = D - 1; a >= 0; --a) {
      int64_t ci = (int64_t)floor((J->x[3 * i + a] - lo[a]) / cs);
      if (ci >= nc[a]) ci = nc[a] - 1;
      c = c * nc[a] + ci;
    }
    cell[i] = c;
    cstart[c + 1]++;
  }
  for (int64_t c = 0; c < ncell; ++c) cstart[c + 1] += cstart[c];
  for (int64_t i = 0; i < n; ++i) bucket[cstart[cell[i]] + fill[cell[i]]++] = i;
  buckets_t B = {{nc[0], nc[1], nc[2]}, cstart, cell, bucket};

  /* count, then offsets, then fill */
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t i = 0; i < n; ++i)
    J->off[i + 1] = ftype(J, i) == T_SI ? 0 : scan_particle(J, &B, i, NULL);
  J->off[0] = 0;
  for (int64_t i = 0; i < n; ++i) J->off[i + 1] += J->off[i];
  int64_t total = J->off[n];
  if (total > J->cap) {
    free(J->nb); free(J->rel);
    J->cap = total + total / 4 + 16;
    J->nb = malloc(sizeof(int32_t) * (size_t)J->cap);
    J->rel = malloc(sizeof(int8_t) * (size_t)J->cap);
    if (!J->nb || !J->rel) {
      free(cstart); free(cell); free(bucket); free(fill);
      set_err("out of memory");
      return -1;
    }
  }
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t i = 0; i < n; ++i) {
    if (ftype(J, i) == T_SI) continue;
    int32_t *out = J->nb + J->off[i];
    int64_t m = scan_particle(J, &B, i, out);
    qsort(out, (size_t)m, sizeof(int32_t), J->P.sum_order ? cmp_i32_desc : cmp_i32);
    for (int64_t t = 0; t < m; ++t) J->rel[J->off[i] + t] = (int8_t)relation(J, i, out[t]);
  }
  free(cstart); free(cell); free(bucket); free(fill);
  return 0;
}

static void compute_h(sphref_job *J) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < J->n; ++i) J->h[i] = h_at(&J->G, &J->S, J->x + 3 * i);
}

int32_t sphref_neighbors(sphref_job *J, int64_t *offsets, int32_t *ids,
                         int8_t *rel_out, int64_t cap, int64_t *n_pairs) {
  compute_h(J);
  if (build_lists(J)) return -1;
  int64_t total = J->off[J->n];
  if (n_pairs) *n_pairs = total;
  if (J->P.sum_order)                       /* report ids ascending regardless */
    for (int64_t i = 0; i < J->n; ++i) {
      int64_t b = J->off[i], e = J->off[i + 1];
      for (int64_t t = 0; t < (e - b) / 2; ++t) {
        int32_t tmp = J->nb[b + t]; J->nb[b + t] = J->nb[e - 1 - t]; J->nb[e - 1 - t] = tmp;
        int8_t tr = J->rel[b + t]; J->rel[b + t] = J->rel[e - 1 - t]; J->rel[e - 1 - t] = tr;
      }
    }
  if (offsets) memcpy(offsets, J->off, sizeof(int64_t) * (size_t)(J->n + 1));
  if (ids || rel_out) {
    if (cap < total) { set_err("capacity too small"); return -1; }
    if (ids) memcpy(ids, J->nb, sizeof(int32_t) * (size_t)total);
    if (rel_out) memcpy(rel_out, J->rel, (size_t)total);
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* control: convergence error, phases, velocity resets (sec. 3.4)        */
/* ------------------------------------------------------------------ */
static int is_moving(const grp_t *g) { return g->phase != PH_FROZEN; }

/* damping factor of the current step (Eq. (momentum_equation_new); reading
 * R20/R21: eps in Phase One, ramped linearly to zero, zero in Phase Two) */
static double damping(const sphref_params *P, const grp_t *g) {
  if (g->phase == PH_ONE) return P->eps_damp;
  if (g->phase == PH_RAMP) return P->eps_damp * (1.0 - (double)g->n_ph / (double)P->ramp_steps);
  return 0.0;
}

/* end-of-step control of one group given this step's V-bar (sum of V~ over the
 * group) and final time step dt.  Sampling and windows follow sec. 3.4.2
 * (V-bar sampled every sample_every phase-local steps, windows of
 * window_samples samples that do not overlap); the phase logic follows
 * sec. 3.4.3-3.4.4 (a time-step drop flagged at the end of a step resets at
 * the start of the next; the transition halves the reset period every
 * ramp_halving steps and lowers the damping linearly). */
static void control_end_of_step(const sphref_params *P, grp_t *g, double vbar, double dt) {
  g->n_ph += 1;
  if (g->n_ph % P->sample_every == 0) {
    g->vbar = vbar;
    g->ring[g->nring++] = vbar;
    if (g->nring == P->window_samples) {
      double s = 0.0;
      for (int q = 0; q < g->nring; ++q) s = s + g->ring[q];
      g->a_prev = g->a_last;
      g->a_last = s / (double)g->nring;
      g->nwin += 1;
      g->nring = 0;
    }
    double et = g->nwin >= 1 ? fabs(vbar - g->a_last) / g->a_last : INFINITY;
    double ea = g->nwin >= 2 ? fabs(g->a_last - g->a_prev) / g->a_prev : INFINITY;
    g->esys = et > ea ? et : ea;
  }
  if (g->phase == PH_ONE) {
    if (g->esys < P->tol || g->n_ph >= P->max_phase1_steps) { g->phase = PH_RAMP; g->n_ph = 0; }
  } else if (g->phase == PH_RAMP) {
    if (g->n_ph >= P->ramp_steps) { g->phase = PH_TWO; g->n_ph = 0; }
  } else if (g->phase == PH_TWO) {
    if (g->n_ph >= P->phase2_steps) g->phase = PH_FROZEN;
  }
  if (g->phase == PH_ONE) {
    g->reset_next = (g->n_ph % P->reset_period == 0) ||
                    (g->dt_prev > 0.0 && dt < 0.1 * g->dt_prev);
  } else if (g->phase == PH_RAMP) {
    int shift = g->n_ph / P->ramp_halving;
    int period = shift >= 30 ? 1 : P->reset_period >> shift;
    if (period < 1) period = 1;
    g->reset_next = g->n_ph % period == 0;
  } else {
    g->reset_next = 1;
  }
  g->dt_prev = dt;
}

int32_t sphref_control_replay(const sphref_params *p, int32_t n_steps,
                              const double *vbar, const double *dt,
                              int32_t *phase_out, int32_t *reset_out,
                              double *esys_out) {
  grp_t g;
  grp_init(&g);
  for (int32_t k = 0; k < n_steps; ++k) {
    if (g.phase != PH_FROZEN) control_end_of_step(p, &g, vbar[k], dt[k]);
    if (phase_out) phase_out[k] = g.phase;
    if (reset_out) reset_out[k] = g.reset_next;
    if (esys_out) esys_out[k] = g.esys;
  }
  return 0;
}


/* Shepard term, particle volume, pressure force with the boundary term,
 * mapped onto the feature (Eqs. (gamma_disc_renormSPH), (particle_volume),
 * (sph_pressure_force_disc_weighted)) of particle i over its list nb / rel */
static void sweep_a_particle(const sphref_job *J, int64_t i, const int32_t *nbl, const int8_t *rel,
                             int64_t cnt, double *ap_out, double *Vt_out, double *gam_out) {
  const geo_t *G = &J->G;
  const sphref_params *P = &J->P;
  int D = G->dim;
  int k = G->f[J->f[i]].k;
  double hi = J->h[i];
  double hik = hpow(hi, k), hi2k = hik * hik;
  double lk = klen(P);                       /* smoothing length per unit h */
  double li = lk * hi;
  double S = sphref_W(k, 0.0, li);          /* self term */
  double gam = sphref_W(k, 0.0, li) * hik;
  double Pi[3] = {0, 0, 0}, B[3] = {0, 0, 0};
  for (int64_t t = 0; t < cnt; ++t) {
    int64_t j = nbl[t];
    double dx[3] = {0, 0, 0};
    for (int a = 0; a < D; ++a) dx[a] = J->x[3 * i + a] - J->x[3 * j + a];
    double r = norm3(dx);
    double hj = J->h[j];
    double hjk = hpow(hj, k), hj2k = hjk * hjk;
    double lij = lk * (0.5 * (hi + hj));
    if (rel[t] == 1) {
      double w = sphref_W(k, r, li);
      S = S + w;
      gam = gam + w * hjk;
      double c = P->p0 * (hi2k + hj2k) * dWdr_over_r(k, r, lij);
      for (int a = 0; a < D; ++a) Pi[a] = Pi[a] + c * dx[a];
    } else {
      /* the particle volume of Eq. (particle_volume) is the inverse of i's
       * number density: every particle that acts on i counts, the boundary
       * particles too */
      S = S + sphref_W(k, r, li);
      double omega = P->boundary_weighting == 0 ? 1.0 / hj
                   : P->boundary_weighting == 1 ? hpow(hj, k - 1) : 0.0;
      omega = omega * bscale(P);
      double nb[3];
      bnormal(G, J->f[i], J->f[j], J->x + 3 * j, J->x + 3 * i, nb);
      double c = P->p0 * (hi2k + hj2k) * sphref_W(k, r, lij) * omega;
      for (int a = 0; a < D; ++a) B[a] = B[a] + c * nb[a];
    }
  }
  double ap[3] = {0, 0, 0};
  for (int a = 0; a < D; ++a) ap[a] = -((Pi[a] + B[a]) / gam);
  tproject(G, J->f[i], J->x + 3 * i, ap);
  for (int a = 0; a < 3; ++a) ap_out[a] = ap[a];
  *Vt_out = 1.0 / S;
  *gam_out = gam;
}


/* h of particle j at the current positions, computed on first use */
static double h_of(sphref_job *J, int64_t j) {
  if (isnan(J->h[j])) J->h[j] = h_at(&J->G, &J->S, J->x + 3 * j);
  return J->h[j];
}

/* Lipschitz constant of h_t: |grad d| <= 1 for the distance to the holes */
static double h_lipschitz(const sphref_sizing *S, int D) {
  if (S->kind == 0) return 0.0;
  if (S->kind == 1 || S->kind == 3) return S->grad;
  if (S->kind == 4) return grid_lipschitz(S, D);
  return S->h0 * S->grad;
}

/* brute_list with h evaluated only where the predicate can hold: with L the
 * Lipschitz constant of h_t, h_j <= h_i + L r, so a j at distance
 * r >= R_i = c h_i / (1 - c L) has c^2 max(h_i, h_j)^2 <= r^2 and is no
 * neighbour (R_i^2 is widened by 1e-9 for rounding).  Same predicate and
 * relation as build_lists; ids ascending. */
static int64_t brute_list_lazy(sphref_job *J, int64_t i, int32_t *ids, int8_t *rel, int64_t cap) {
  int64_t c = 0;
  if (ftype(J, i) == T_SI) return 0;
  int D = J->G.dim;
  double hi = h_of(J, i);
  double L = h_lipschitz(&J->S, J->G.dim);
  double R2 = INFINITY;
  double cr = rc_ratio(&J->P);
  if (cr * L < 1.0) { double R = cr * hi / (1.0 - cr * L); R2 = R * R * (1.0 + 1e-9); }
  for (int64_t j = 0; j < J->n; ++j) {
    if (j == i) continue;
    double s = 0.0;
    for (int a = 0; a < D; ++a) {
      double d = J->x[3 * i + a] - J->x[3 * j + a];
      s = s + d * d;
    }
    if (!(s < R2)) continue;
    double hj = h_of(J, j);
    double m = hi > hj ? hi : hj;
    if (!(s < (cr * cr) * (m * m))) continue;
    int r = relation(J, i, j);
    if (!r) continue;
    if (c < cap) { ids[c] = (int32_t)j; rel[c] = (int8_t)r; }
    c++;
  }
  return c;
}

int32_t sphref_sample(sphref_job *J, int32_t m, const int64_t *idx, int64_t *offsets,
                      int32_t *ids, int8_t *rel, int64_t cap, double *ap, double *vt,
                      double *gam) {
  for (int64_t j = 0; j < J->n; ++j) J->h[j] = NAN;   /* h at the current positions, lazily */
  int64_t total = 0;
  offsets[0] = 0;
  for (int32_t s = 0; s < m; ++s) {
    int64_t i = idx[s];
    if (i < 0 || i >= J->n) { set_err("sample index out of range"); return -1; }
    int64_t c = brute_list_lazy(J, i, ids + total, rel + total, cap - total);
    if (total + c > cap) { set_err("capacity too small"); return -1; }
    if (ftype(J, i) != T_SI)
      sweep_a_particle(J, i, ids + total, rel + total, c, ap + 3 * s, vt + s, gam + s);
    else {
      ap[3 * s] = ap[3 * s + 1] = ap[3 * s + 2] = 0.0;
      vt[s] = gam[s] = 0.0;
    }
    total += c;
    offsets[s + 1] = total;
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* one relaxation step (Algorithm 1; every feature reads x^n, and the  */
/* force is evaluated once per step, see the integration below)         */
/* ------------------------------------------------------------------ */

/* Eq. (fa_time_step_size) terms of one particle folded into a running min;
 * r_c = c h, nu = 0.1 r_c |v|.  Infinite terms (a or v zero) drop out. */
static double dt_terms(double dt, double cr, double h, double amag, double vmag) {
  double rc = cr * h;
  if (amag > 0.0) { double t = 0.25 * sqrt(rc / amag); if (t < dt) dt = t; }
  if (vmag > 0.0) {
    double t = rc / (40.0 * vmag);
    if (t < dt) dt = t;
    double nu = 0.1 * rc * vmag;
    t = 0.125 * rc * rc / nu;
    if (t < dt) dt = t;
  }
  return dt;
}

static int one_step(sphref_job *J) {
  const geo_t *G = &J->G;
  const sphref_params *P = &J->P;
  int D = G->dim;
  int64_t n = J->n;

  /* targets h_i = h_t(x_i^n); lists over x^n */
  compute_h(J);
  if (build_lists(J)) return -1;

  /* which particles evolve this step: not singular, group not converged
   * (Algorithm 1: "if V-bar_{*,k} is not converged") */
  char *act = malloc((size_t)(n > 0 ? n : 1));
  if (!act) { set_err("out of memory"); return -1; }
  for (int64_t i = 0; i < n; ++i) act[i] = ftype(J, i) != T_SI && is_moving(&J->g[J->f[i]]);

  /* reset forces; reset velocities of groups flagged at the previous step */
  for (int64_t i = 0; i < 3 * n; ++i) { J->ap[i] = 0.0; J->a[i] = 0.0; J->vt[i] = 0.0; }
  for (int64_t i = 0; i < n; ++i) { J->Vt[i] = 0.0; J->gam[i] = 0.0; J->eta[i] = 0.0; }
  for (int64_t i = 0; i < n; ++i)
    if (act[i] && J->g[J->f[i]].reset_next)
      for (int a = 0; a < 3; ++a) J->v[3 * i + a] = 0.0;

  int64_t inter = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : inter)
  for (int64_t i = 0; i < n; ++i) {
    if (!act[i]) continue;
    int64_t cnt = J->off[i + 1] - J->off[i];
    inter += cnt;
    sweep_a_particle(J, i, J->nb + J->off[i], J->rel + J->off[i], cnt, J->ap + 3 * i, &J->Vt[i],
                     &J->gam[i]);
  }

  /* first time step per group from a^p and v^n */
  for (int q = 0; q < G->nf; ++q) J->g[q].dt1 = P->dt_max;
  for (int64_t i = 0; i < n; ++i) {
    if (!act[i]) continue;
    grp_t *g = &J->g[J->f[i]];
    g->dt1 = dt_terms(g->dt1, rc_ratio(P), J->h[i], norm3(J->ap + 3 * i), norm3(J->v + 3 * i));
  }

  /* mid-point velocity */
  for (int64_t i = 0; i < n; ++i) {
    if (!act[i]) continue;
    double dt1 = J->g[J->f[i]].dt1;
    for (int a = 0; a < D; ++a) J->vt[3 * i + a] = J->v[3 * i + a] + 0.5 * dt1 * J->ap[3 * i + a];
  }

  /* viscous force with the mid-point velocity (nu_i = 0.1 r_c |v~_i| per
   * particle, combined by the harmonic mean of eta) */
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    if (!act[i]) continue;
    int k = G->f[J->f[i]].k;
    double nu = 0.1 * (rc_ratio(P) * J->h[i]) * norm3(J->vt + 3 * i);
    J->eta[i] = nu / hpow(J->h[i], k);         /* eta = rho_t nu, rho_t = h^-k */
  }
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t i = 0; i < n; ++i) {
    if (!act[i]) continue;
    int k = G->f[J->f[i]].k;
    double hi = J->h[i];
    double hik = hpow(hi, k), hi2k = hik * hik;
    double Fv[3] = {0, 0, 0};
    for (int64_t t = J->off[i]; t < J->off[i + 1]; ++t) {
      if (J->rel[t] != 1) continue;
      int64_t j = J->nb[t];
      double dx[3] = {0, 0, 0};
      for (int a = 0; a < D; ++a) dx[a] = J->x[3 * i + a] - J->x[3 * j + a];
      double r = norm3(dx);
      double hj = J->h[j];
      double hjk = hpow(hj, k), hj2k = hjk * hjk;
      double es = J->eta[i] + J->eta[j];
      double H = es > 0.0 ? 2.0 * J->eta[i] * J->eta[j] / es : 0.0;
      double c = H * (hi2k + hj2k) * dWdr_over_r(k, r, klen(P) * (0.5 * (hi + hj)));
      for (int a = 0; a < D; ++a) Fv[a] = Fv[a] + c * (J->vt[3 * i + a] - J->vt[3 * j + a]);
    }
    tproject(G, J->f[i], J->x + 3 * i, Fv);
    double eps = damping(P, &J->g[J->f[i]]);
    for (int a = 0; a < D; ++a)
      J->a[3 * i + a] = J->ap[3 * i + a] + Fv[a] - eps * J->v[3 * i + a];
  }

  /* final time step per group from a and v~ */
  for (int q = 0; q < G->nf; ++q) J->g[q].dt = P->dt_max;
  for (int64_t i = 0; i < n; ++i) {
    if (!act[i]) continue;
    grp_t *g = &J->g[J->f[i]];
    g->dt = dt_terms(g->dt, rc_ratio(P), J->h[i], norm3(J->a + 3 * i), norm3(J->vt + 3 * i));
  }

  /* integrate and map onto the feature.  Algorithm 1 updates, in order, the
   * mid-point velocity v~ = v^n + dt1 a^p / 2 (formed above, cited Eq. 26),
   * the predicted velocity v^(n+1/2) = v^n + dt a / 2 (cited Eq. 27) and the
   * position x* = x^n + dt v^(n+1/2) (cited Eq. 28), then maps x* onto the
   * feature; it lists no further velocity update, so the velocity carried
   * into the next step is v^(n+1/2), tangent to the feature at x^(n+1) */
  int64_t escaped = 0, nonfinite = 0;
#pragma omp parallel for schedule(static) reduction(+ : escaped, nonfinite)
  for (int64_t i = 0; i < n; ++i) {
    if (!act[i]) continue;
    double dt = J->g[J->f[i]].dt;
    double vh[3] = {0, 0, 0}, xs[3] = {0, 0, 0};
    int finite = 1;
    for (int a = 0; a < D; ++a) {
      vh[a] = J->v[3 * i + a] + 0.5 * dt * J->a[3 * i + a];
      xs[a] = J->x[3 * i + a] + dt * vh[a];
      if (!isfinite(xs[a])) finite = 0;
    }
    if (!finite) { nonfinite++; continue; }  /* the job stops after this step */
    int type = ftype(J, i);
    if (type == T_V) {
      if (!inside(G, xs)) {                  /* rejected move: stays, velocity zeroed */
        for (int a = 0; a < 3; ++a) J->v[3 * i + a] = 0.0;
        escaped++;
        continue;
      }
    } else {
      pproject(G, J->f[i], xs);
    }
    double vn[3] = {0, 0, 0};
    for (int a = 0; a < D; ++a) vn[a] = vh[a];
    tproject(G, J->f[i], xs, vn);
    for (int a = 0; a < D; ++a) { J->x[3 * i + a] = xs[a]; J->v[3 * i + a] = vn[a]; }
  }
  J->escaped += escaped;
  if (nonfinite) { J->state_error = 1; set_err("non-finite position"); free(act); return -2; }

  /* V-bar per group and the control law */
  double vbar[MAXF];
  for (int q = 0; q < G->nf; ++q) vbar[q] = 0.0;
  for (int64_t i = 0; i < n; ++i) if (act[i]) vbar[J->f[i]] = vbar[J->f[i]] + J->Vt[i];
  for (int q = 0; q < G->nf; ++q) {
    grp_t *g = &J->g[q];
    if (G->f[q].type == T_SI || g->count == 0 || !is_moving(g)) continue;
    control_end_of_step(P, g, vbar[q], g->dt);
  }
  J->steps++;
  J->inter_last = inter;
  J->inter_total += inter;
  free(act);
  return 0;
}

static int all_frozen(const sphref_job *J) {
  for (int q = 0; q < J->G.nf; ++q)
    if (J->G.f[q].type != T_SI && J->g[q].count > 0 && J->g[q].phase != PH_FROZEN) return 0;
  return 1;
}

int32_t sphref_step(sphref_job *J, int32_t n_steps) {
  if (J->state_error) { set_err("job is in an error state"); return -2; }
  for (int32_t s = 0; s < n_steps; ++s) {
    if (all_frozen(J)) break;
    int rc = one_step(J);
    if (rc) return rc;
  }
  return 0;
}

int32_t sphref_error(sphref_job *J, double *e_sys, int32_t *phase,
                     int32_t *converged, int64_t *step) {
  double e = 0.0;
  int ph = PH_FROZEN, any = 0;
  for (int q = 0; q < J->G.nf; ++q) {
    const grp_t *g = &J->g[q];
    if (J->G.f[q].type == T_SI || g->count == 0) continue;
    any = 1;
    if (g->esys > e || isnan(g->esys)) e = g->esys;
    if (g->phase < ph) ph = g->phase;
  }
  if (!any) { e = 0.0; ph = PH_FROZEN; }
  if (e_sys) *e_sys = e;
  if (phase) *phase = ph;
  if (converged) *converged = all_frozen(J);
  if (step) *step = J->steps;
  return 0;
}

int32_t sphref_group_state(sphref_job *J, int32_t f, double *out) {
  if (f < 0 || f >= J->G.nf) { set_err("bad feature"); return -1; }
  const grp_t *g = &J->g[f];
  out[0] = g->phase; out[1] = g->n_ph; out[2] = g->esys; out[3] = g->dt1; out[4] = g->dt;
  out[5] = g->vbar; out[6] = g->reset_next; out[7] = g->a_last; out[8] = g->a_prev; out[9] = g->nwin;
  return 0;
}

int32_t sphref_counters(sphref_job *J, double *out) {
  out[0] = (double)J->steps;
  out[1] = (double)J->escaped;
  out[2] = (double)J->inter_total;
  out[3] = (double)J->inter_last;
  return 0;
}

/* ------------------------------------------------------------------ */
/* the tag system of the background grid (sec. 3.2): cell types and     */
/* feature indices of a level-set domain                                */
/* ------------------------------------------------------------------ */
enum { C_NEG = 0, C_POS = 1, C_SURF = 2, C_CURVE = 3, C_SING = 4 };

/* cell of point x (clamped to the grid), as (i, j, k) */
static void tag_cell_of(const geo_t *G, const int *nc, const double *x, int *ijk) {
  for (int a = 0; a < 3; ++a) {
    ijk[a] = 0;
    if (a >= G->dim) continue;
    double s = (double)(G->pn[a] - 1) / (G->phi_hi[a] - G->plo[a]);
    double u = floor((x[a] - G->plo[a]) * s);
    if (!(u > 0.0)) u = 0.0;
    if (u > (double)(nc[a] - 1)) u = (double)(nc[a] - 1);
    ijk[a] = (int)u;
  }
}

/* give cell (i, j, k) type t and index v unless a cell of that type already
 * holds it; curve marks do not replace corner marks */
static void tag_mark(int32_t *ctype, int32_t *cindex, const int *nc, int i, int j, int k,
                     int t, int v) {
  if (i < 0 || j < 0 || k < 0 || i >= nc[0] || j >= nc[1] || k >= nc[2]) return;
  int64_t id = ((int64_t)k * nc[1] + j) * nc[0] + i;
  if (ctype[id] == C_SING || (ctype[id] == C_CURVE && t == C_CURVE)) return;
  ctype[id] = t;
  cindex[id] = v;
}

/* number the face-connected components of the cells of type t in the order
 * of their first cell; returns their count */
static int tag_components(int32_t *ctype, int32_t *cindex, const int *nc, int t, int64_t *stack) {
  int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
  int count = 0;
  for (int64_t s = 0; s < ncell; ++s) {
    if (ctype[s] != t || cindex[s] >= 0) continue;
    int64_t top = 0;
    stack[top++] = s;
    cindex[s] = count;
    while (top > 0) {
      int64_t id = stack[--top];
      int i = (int)(id % nc[0]), j = (int)((id / nc[0]) % nc[1]), k = (int)(id / ((int64_t)nc[0] * nc[1]));
      const int off[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
      for (int q = 0; q < 6; ++q) {
        int a = i + off[q][0], b = j + off[q][1], c = k + off[q][2];
        if (a < 0 || b < 0 || c < 0 || a >= nc[0] || b >= nc[1] || c >= nc[2]) continue;
        int64_t nb = ((int64_t)c * nc[1] + b) * nc[0] + a;
        if (ctype[nb] != t || cindex[nb] >= 0) continue;
        cindex[nb] = count;
        stack[top++] = nb;
      }
    }
    ++count;
  }
  return count;
}

int32_t sphref_tags(const sphref_geometry *g, int32_t *ctype, int32_t *cindex,
                    int32_t *n_volumes, int32_t *n_patches, int32_t *curve_patches) {
  /* the patches are what this finds: a 3D geometry may leave them unset */
  geo_t G;
  sphref_geometry gg;
  int32_t *unset = NULL;
  if (g && g->dim == 3 && g->n_curves > 0 && (g->n_patches < 1 || !g->curve_patches)) {
    gg = *g;
    unset = malloc(2 * (size_t)g->n_curves * sizeof(int32_t));
    if (!unset) { set_err("out of memory"); return -1; }
    for (int q = 0; q < 2 * g->n_curves; ++q) unset[q] = -1;
    gg.n_patches = 1;
    gg.curve_patches = unset;
    g = &gg;
  }
  int bad = geo_build(g, &G);
  free(unset);
  if (bad) return -1;
  if (G.domain != 2) { set_err("the tag system needs a level-set domain"); return -1; }
  if (!ctype || !cindex || !n_volumes || !n_patches || (G.ncv > 0 && !curve_patches)) {
    set_err("bad argument"); return -1;
  }
  int D = G.dim, nc[3] = {1, 1, 1};
  for (int a = 0; a < D; ++a) nc[a] = G.pn[a] - 1;
  int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
  /* phi at the cell's nodes: all positive, all negative, or mixed */
  for (int k = 0; k < nc[2]; ++k)
    for (int j = 0; j < nc[1]; ++j)
      for (int i = 0; i < nc[0]; ++i) {
        int pos = 0, neg = 0, nn = D == 3 ? 8 : 4;
        for (int q = 0; q < nn; ++q) {
          int a = i + (q & 1), b = j + ((q >> 1) & 1), c = k + ((q >> 2) & 1);
          double v = G.phi[((int64_t)c * G.pn[1] + b) * G.pn[0] + a];
          pos += v > 0.0;
          neg += v < 0.0;
        }
        int64_t id = ((int64_t)k * nc[1] + j) * nc[0] + i;
        ctype[id] = pos == nn ? C_POS : (neg == nn ? C_NEG : C_SURF);
        cindex[id] = -1;
      }
  /* curves: the cells of points along each segment, a quarter of the
   * smallest cell side apart, and their face neighbours */
  double side = INFINITY;
  for (int a = 0; a < D; ++a) {
    double w = (G.phi_hi[a] - G.plo[a]) / (double)nc[a];
    if (w < side) side = w;
  }
  for (int c = 0; c < G.ncv; ++c)
    for (int s = G.coff[c]; s + 1 < G.coff[c + 1]; ++s) {
      const double *p0 = G.cpts + 3 * s, *p1 = p0 + 3;
      double e[3] = {0, 0, 0}, l2 = 0.0;
      for (int a = 0; a < D; ++a) { e[a] = p1[a] - p0[a]; l2 = l2 + e[a] * e[a]; }
      int64_t ns = (int64_t)ceil(sqrt(l2) / (0.25 * side));
      if (ns < 1) ns = 1;
      for (int64_t q = 0; q <= ns; ++q) {
        double x[3] = {0, 0, 0}, tq = (double)q / (double)ns;
        for (int a = 0; a < D; ++a) x[a] = p0[a] + tq * e[a];
        int ijk[3];
        tag_cell_of(&G, nc, x, ijk);
        tag_mark(ctype, cindex, nc, ijk[0], ijk[1], ijk[2], C_CURVE, c);
        for (int a = 0; a < D; ++a)
          for (int sd = -1; sd <= 1; sd += 2) {
            int o[3] = {ijk[0], ijk[1], ijk[2]};
            o[a] += sd;
            tag_mark(ctype, cindex, nc, o[0], o[1], o[2], C_CURVE, c);
          }
      }
    }
  /* corners: their cell and all its neighbours */
  for (int m = 0; m < G.ncr; ++m) {
    int ijk[3];
    tag_cell_of(&G, nc, G.cor[m], ijk);
    for (int dk = (D == 3 ? -1 : 0); dk <= (D == 3 ? 1 : 0); ++dk)
      for (int dj = -1; dj <= 1; ++dj)
        for (int di = -1; di <= 1; ++di) {
          int i = ijk[0] + di, j = ijk[1] + dj, k = ijk[2] + dk;
          if (i < 0 || j < 0 || k < 0 || i >= nc[0] || j >= nc[1] || k >= nc[2]) continue;
          int64_t id = ((int64_t)k * nc[1] + j) * nc[0] + i;
          if (ctype[id] == C_SING) continue;
          ctype[id] = C_SING;
          cindex[id] = m;
        }
  }
  int64_t *stack = malloc((size_t)ncell * sizeof(int64_t));
  if (!stack) { set_err("out of memory"); return -1; }
  *n_patches = tag_components(ctype, cindex, nc, C_SURF, stack);
  *n_volumes = tag_components(ctype, cindex, nc, C_POS, stack);
  free(stack);
  /* the patches beside each curve: face neighbours of its cells */
  for (int c = 0; c < G.ncv; ++c) {
    int found[3] = {-1, -1, -1}, nfound = 0;
    for (int64_t id = 0; id < ncell; ++id) {
      if (ctype[id] != C_CURVE || cindex[id] != c) continue;
      int i = (int)(id % nc[0]), j = (int)((id / nc[0]) % nc[1]), k = (int)(id / ((int64_t)nc[0] * nc[1]));
      for (int a = 0; a < D; ++a)
        for (int sd = -1; sd <= 1; sd += 2) {
          int o[3] = {i, j, k};
          o[a] += sd;
          if (o[a] < 0 || o[a] >= nc[a]) continue;
          int64_t nb = ((int64_t)o[2] * nc[1] + o[1]) * nc[0] + o[0];
          if (ctype[nb] != C_SURF) continue;
          int p = cindex[nb], seen = 0;
          for (int q = 0; q < nfound && q < 3; ++q) seen |= found[q] == p;
          if (!seen) {
            if (nfound < 3) found[nfound] = p;
            ++nfound;
          }
        }
    }
    if (nfound > 2) {
      curve_patches[2 * c] = -2;
      curve_patches[2 * c + 1] = -1;
      continue;
    }
    if (nfound == 2 && found[1] < found[0]) { int t = found[0]; found[0] = found[1]; found[1] = t; }
    curve_patches[2 * c] = found[0];
    curve_patches[2 * c + 1] = found[1];
  }
  return 0;
}
