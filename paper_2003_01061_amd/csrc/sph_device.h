// sph_device.h -- device-side data layout and math of the feature-aware SPH
// relaxation step for gfx950 (CDNA4, wave64).
//
// Layout in HBM: particles sit in cell order as packed 32-byte records, one
// array of {x, y, z, h} (FP64, z = 0 in 2D) and one of {vx, vy, vz, 0}
// (FP64), so a neighbour gather touches one 32-byte sector per record; the
// feature index is a u16 and the caller's id a u32 column.  Accelerations
// are {ax, ay, az, 0} records in the sweep precision.  The neighbour list is
// blocked ELL: entries 8b .. 8b+7 of slot i form one 32-byte block at words
// [(b * n + i) * 8, +8), so a lane appends whole 32-byte sectors and the 64
// lanes of a wave reading block b touch 2 KB of consecutive memory.  The top
// bit of an entry marks a boundary neighbour (a lower-dimensional feature
// bounding the particle's own, paper sec. 3.3), the low 31 bits are the slot.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sph {

constexpr int LB = 8;           // neighbour-list entries per block (32 bytes)
constexpr int MAXF = 64;        // features per job; a job's features own ids [64 s, 64 s + nf)
constexpr int MAXJ = 64;        // jobs per batch
constexpr int MAXH = 16;        // holes per job
constexpr int MAXRING = 64;     // samples per averaging window
constexpr int BLOCK = 256;
constexpr int NSTRIPE = 64;     // copies of each atomic accumulator (spreads contention)

// tuning knobs (compile time): entries of a particle's neighbour list the
// neighbour kernel keeps in LDS for its pair sums (a multiple of LB; 256
// threads x 32 x 4 bytes = 32 KB per block), records loaded together per
// neighbour batch, and whether blocks are remapped so that each XCD gets a
// contiguous range
#ifndef SPH_LDS_LIST
#define SPH_LDS_LIST 32
#endif
#ifndef SPH_NBATCH
#define SPH_NBATCH 4
#endif
static_assert(SPH_NBATCH >= 1 && SPH_NBATCH <= 8, "records are padded by 8");
#ifndef SPH_GBATCH
#define SPH_GBATCH 4
#endif
// lanes per particle of the FP32 Verlet filter-and-sweep kernel in 3D (1 or
// 2; 2D keeps one: its short lists do not pay for the per-particle work that
// both lanes repeat)
// lanes per particle of the 3D viscous sweep (1 or 2)
#ifndef SPH_SWEEPB_LANES
#define SPH_SWEEPB_LANES 2
#endif
#ifndef SPH_VERLET_LANES
#define SPH_VERLET_LANES 2
#endif
#ifndef SPH_XCD_REMAP
#define SPH_XCD_REMAP 1
#endif

enum : int { T_SI = 0, T_C = 1, T_S = 2, T_V = 3 };
enum : int { K_VOL = 0, K_BOXSIDE = 1, K_HOLE = 2, K_EDGE3 = 3, K_CORNER = 4, K_SHELL = 5,
              K_LEVEL = 6, K_POLY = 7, K_PCORNER = 8 };
enum : int { PH_ONE = 1, PH_RAMP = 2, PH_TWO = 3, PH_FROZEN = 4 };

// one feature: the paper's (type, index) pair and what its geometry is
struct Feat {
  int8_t type, k, kind, axis, side, fax0, fsd0, fax1, fsd1, hole, bits, pad[5];
};

// outward normal n_b of feature fi's boundary at a particle of feature fb
// (paper sec. 3.3): mode 0 no relation, 1 the constant vector n; 2 (a ball
// hole), 3 (an ellipsoidal hole), 4 (the ball domain's sphere), 5 (the zero
// level set) and 6 (an imported curve) the particle's own normal out of the
// domain, which k_rank_gather stores; 7 (a 3D patch at a curve beside it) and
// 8 (at a vertex) depend on the pair and are computed in the sweep
struct BNorm {
  int32_t mode, hole;
  double n[3];
};

struct Geom {
  int32_t dim, nf, nh, hkind;
  double lo[3], hi[3];
  double hc[MAXH][3];
  double hr[MAXH];
  double h0, grad, dcap, hpt[3];
  int32_t hell[MAXH];       // 1: ellipsoidal hole (unequal semi-axes)
  double ha[MAXH][3];       // its semi-axes, and max over them
  double hamax[MAXH], hamin[MAXH];   // largest / smallest semi-axis of an ellipsoid
  double hR[MAXH][9];       // rotation, row-major: local y = R (x - c)
  int32_t domain, pad;      // 0 box minus holes, 1 the ball inscribed in the box
  double dc[3], dR;         // ball domain: centre and radius
  const double *grid;       // gridded sizing: node values (device), x fastest
  int32_t gn[3], gpad;      // nodes per axis
  double glo[3], gs[3];     // grid origin and (n - 1) / (hi - lo) per axis
  const double *phi;        // level-set domain: node values (device), x fastest
  int32_t pn[3], ppad;
  double plo[3], ps[3];
  const double *cpts;       // imported curves: points (x, y, z per point, device)
  const int32_t *coff;      // curve c owns the points [coff[c], coff[c + 1])
};

// imported curve c (a polyline; in 2D with the domain on its left): the
// segment whose closest point to x is nearest (the first on ties), that
// point in q (D components)
template <int D>
__host__ __device__ __forceinline__ int poly_closest(const Geom &g, int c, const double *x, double *q) {
  // start from the first point, so that a segment is returned even when no
  // distance compares (a non-finite x)
  int best = g.coff[c];
  for (int a = 0; a < D; ++a) q[a] = g.cpts[3 * best + a];
  double bd = __builtin_inf();
  for (int k = g.coff[c]; k + 1 < g.coff[c + 1]; ++k) {
    const double *p0 = g.cpts + 3 * k, *p1 = g.cpts + 3 * (k + 1);
    const double e0 = p1[0] - p0[0], e1 = p1[1] - p0[1], e2 = D == 3 ? p1[2] - p0[2] : 0.0;
    const double ee = D == 3 ? e0 * e0 + e1 * e1 + e2 * e2 : e0 * e0 + e1 * e1;
    const double xe = D == 3 ? (x[0] - p0[0]) * e0 + (x[1] - p0[1]) * e1 + (x[2] - p0[2]) * e2
                             : (x[0] - p0[0]) * e0 + (x[1] - p0[1]) * e1;
    double t = ee > 0.0 ? xe / ee : 0.0;
    t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
    const double c0 = p0[0] + t * e0, c1 = p0[1] + t * e1, c2 = D == 3 ? p0[2] + t * e2 : 0.0;
    const double d0 = x[0] - c0, d1 = x[1] - c1, d2 = D == 3 ? x[2] - c2 : 0.0;
    const double d = D == 3 ? d0 * d0 + d1 * d1 + d2 * d2 : d0 * d0 + d1 * d1;
    if (d < bd) {
      bd = d;
      best = k;
      q[0] = c0;
      q[1] = c1;
      if (D == 3) q[D - 1] = c2;
    }
  }
  return best;
}

// unit tangent of segment k of the imported curves (D components)
template <int D>
__host__ __device__ __forceinline__ void seg_tangent(const Geom &g, int k, double *t) {
  const double *p0 = g.cpts + 3 * k, *p1 = g.cpts + 3 * (k + 1);
  const double e0 = p1[0] - p0[0], e1 = p1[1] - p0[1], e2 = D == 3 ? p1[2] - p0[2] : 0.0;
  const double l = __builtin_sqrt(D == 3 ? e0 * e0 + e1 * e1 + e2 * e2 : e0 * e0 + e1 * e1);
  t[0] = e0 / l;
  t[1] = e1 / l;
  if (D == 3) t[D - 1] = e2 / l;
}

// the gridded level set of a level-set domain: phi multilinear in the grid
// cell of x (coordinates clamped to the grid box), and its gradient, the
// derivative of that multilinear function in the cell
template <int D>
__host__ __device__ __forceinline__ double ls_phi(const Geom &g, const double *x, double *gr) {
#pragma clang fp contract(off)
  int c[3] = {0, 0, 0};
  double t[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < D; ++a) {
    const double top = (double)(g.pn[a] - 1);
    double u = (x[a] - g.plo[a]) * g.ps[a];
    u = u > 0.0 ? u : 0.0;
    u = u < top ? u : top;
    double f = __builtin_floor(u);
    f = f < top - 1.0 ? f : top - 1.0;
    c[a] = (int)f;
    t[a] = u - f;
  }
  const int nx = g.pn[0], ny = g.pn[1];
  double v[2][2], d[2][2];
  for (int dz = 0; dz < (D == 3 ? 2 : 1); ++dz)
    for (int dy = 0; dy < 2; ++dy) {
      const long long row = ((long long)(c[2] + dz) * ny + (c[1] + dy)) * nx + c[0];
      const double g0 = g.phi[row], g1 = g.phi[row + 1];
      d[dz][dy] = g1 - g0;
      v[dz][dy] = g0 + t[0] * d[dz][dy];
    }
  double w[2], e[2], q[2];
  for (int dz = 0; dz < (D == 3 ? 2 : 1); ++dz) {
    q[dz] = v[dz][1] - v[dz][0];
    w[dz] = v[dz][0] + t[1] * q[dz];
    e[dz] = d[dz][0] + t[1] * (d[dz][1] - d[dz][0]);
  }
  gr[0] = gr[1] = gr[2] = 0.0;
  if (D == 2) {
    gr[0] = g.ps[0] * e[0];
    gr[1] = g.ps[1] * q[0];
    return w[0];
  }
  gr[0] = g.ps[0] * (e[0] + t[2] * (e[1] - e[0]));
  gr[1] = g.ps[1] * (q[0] + t[2] * (q[1] - q[0]));
  gr[2] = g.ps[2] * (w[1] - w[0]);
  return w[0] + t[2] * (w[1] - w[0]);
}

// unit normal of the level set towards increasing phi (0 where grad vanishes)
template <int D>
__host__ __device__ __forceinline__ void ls_unit(const Geom &g, const double *x, double *m) {
  double gr[3];
  (void)ls_phi<D>(g, x, gr);
  double s = 0.0;
  for (int a = 0; a < D; ++a) s += gr[a] * gr[a];
  const double r = __builtin_sqrt(s);
  m[0] = m[1] = m[2] = 0.0;
  if (!(r > 0.0)) return;
  for (int a = 0; a < D; ++a) m[a] = gr[a] / r;
}

// uniform cell grid over a job's box; its cells own the global cell ids
// [cbase, cbase + ncell) of the batch; per-particle search radius
// R_i = min(rfac h_i, rmax) (rfac from the Lipschitz bound of h_t)
// A job's cells: nlev uniform grids over its box, one per band of h
// (level l holds the particles with hthr[l] <= h < hthr[l+1], cell side
// ~ 2 hthr[l] cell_factor), laid end to end from cbase (level l from
// cbase + lbase[l]).  One level is the plain uniform grid.
constexpr int MAXLEV = 6;
struct Grid {
  int32_t nlev;
  uint32_t ncell, cbase;
  uint32_t lbase[MAXLEV];
  int32_t nc[MAXLEV][3];
  double lo[3];
  double inv_c[MAXLEV][3], c[MAXLEV][3];
  double hthr[MAXLEV];   // lower h bound of level l (hthr[0] = 0)
  double hcap[MAXLEV];   // h of a level-l particle is below hcap[l] (the last: <= h_max)
  double cmax;           // largest cell side over the levels
  double rfac, rmax, lip;
};

struct Ctl {
  double tol, eps_damp, dt_max;
  int32_t reset_period, sample_every, window_samples, ramp_steps, ramp_halving,
      phase2_steps, max_phase1_steps, pad;
};

// per-feature group: inputs of the coming step, accumulators of the running
// step (order independent: min of non-negative double bit patterns, integer
// fixed-point sums), and the control state of sec. 3.4
struct Group {
  int32_t active, reset_now;
  double eps;
  unsigned long long dt1_bits, dt_bits, vsum;
  int32_t phase, n_ph, nring, nwin, count, tracked, reset_next, pad;
  double vscale, dt_prev, dt1, dt, esys, vbar, a_last, a_prev;
  double ring[MAXRING];
};

// per-job counters and error flags
struct JobStat {
  unsigned long long escaped, inter_total, inter_last, steps;
  unsigned int nan_flag, nan_oid, overflow, overflow_max;
  unsigned int skin_overflow, skin_max;   // the Verlet candidate list's overflow
  int32_t converged, live;
};

struct JobDev {
  Geom g;
  Grid G;
  Ctl ctl;
  double p0;
  // cut-off radius r_c = ksup h; the kernel's smoothing length is klen h
  // (klen = ksup / 2) and the pair predicate compares with ksup2 max(h)^2
  double ksup, klen, ksup2;
  double iband;    // 1 / (2 klen h0): the FP32 band's rounding bound per unit of M
  double bscale;   // factor on the boundary term of the pressure force
  // Verlet candidate list (skin delta h): its reach ksup_s = ksup + delta, the
  // scan radius factor and cap at that reach, and the displacement since the
  // list's build, in units of the particle's h then, that forces a rebuild
  double ksup_s, rfac_s, rmax_s, move_eps;
  int32_t bw, nf, live;
  int32_t vol;   // the job's volume feature (local id), -1 if none
};

struct Parts {
  double4 *xh;      // x, y, z, h
  double4 *v;       // vx, vy, vz, 0
  uint16_t *f;      // global feature id = 64 * job slot + local feature
  uint32_t *oid;    // caller's id inside the job
  float4 *xf;       // the neighbour scan's FP32 record: {x, y, h, feature bits} in
                    // 2D; {x, y, z, h'} in 3D, h' = h rounded to FP32 with its 6
                    // low mantissa bits replaced by the job-local feature id
};

// FP32 scan record of a particle (the rounding of its FP64 record)
template <int D>
__device__ __forceinline__ float4 scan_record(const double4 &xh, uint32_t f) {
  // 2h (scaling by 2 commutes with the rounding); the support radius is
  // klen 2h
  if (D == 2) return make_float4((float)xh.x, (float)xh.y, (float)(2.0 * xh.w), __uint_as_float(f));
  const uint32_t hb =
      (__float_as_uint((float)(2.0 * xh.w)) & ~(uint32_t)(MAXF - 1)) | (f & (MAXF - 1));
  return make_float4((float)xh.x, (float)xh.y, (float)xh.z, __uint_as_float(hb));
}

// tables and accumulators shared by every kernel of a batch
struct Batch {
  const JobDev *jobs;                 // [MAXJ]
  const Feat *feat;                   // [MAXJ * MAXF]
  const unsigned long long *bmask;    // [MAXJ * MAXF] bit l: local feature l bounds this one
  const BNorm *bn;                    // [MAXJ * MAXF][MAXF]
  Group *grp;                         // [MAXJ * MAXF]
  JobStat *st;                        // [MAXJ]
  unsigned int *gflags;               // [0] a scan tile gave up waiting (never expected)
  unsigned long long *smin, *ssum;    // [MAXJ * MAXF][NSTRIPE] group minima / sums
  unsigned long long *scnt, *sesc;    // [MAXJ][NSTRIPE] interactions / rejected moves
  double4 *enrm;                      // [n] cell order: for a particle of a feature of
                                      // lower dimension than the domain, the domain's outward
                                      // normal there (k_rank_gather)
  int n, cap;
  uint32_t ncell, ntiles;
  int njobs;                          // job slots in use: [0, njobs)
  // Verlet candidate lists (skin_on): built when vstate[VS_REBUILD] is set,
  // filtered into the neighbour list every step; particles keep their slots
  // between builds
  int skin_on, skin_cap;
  uint32_t *skin, *nsk;               // [skin_cap / 8][n][8] blocked like the list; counts
  double4 *xref;                      // [n] x and h at the last build
  unsigned long long *vstate;         // [VS_REBUILD] the rebuild flag, [VS_BUILDS]
                                      // builds so far, [VS_TRIP] set by the
                                      // integration when a particle moved too far
};
constexpr int VS_REBUILD = 0, VS_BUILDS = 1, VS_TRIP = 2, VS_WORDS = 3;

template <typename R>
struct Vec4;
template <>
struct Vec4<float> {
  using T = float4;
};
template <>
struct Vec4<double> {
  using T = double4;
};

// ---------------------------------------------------------------------------
// exact FP64 pieces shared by the neighbour predicate and the sizing function
// ---------------------------------------------------------------------------

// h_t(x) of the sizing record: squared distances summed over axes in order,
// sqrt, no fused multiply-add, so that it is bit-reproducible.
// ---------------------------------------------------------------------------
// ellipsoidal holes: sum_k (y_k / a_k)^2 <= 1 with y = R (x - c).  The
// operations that decide h and the inside test run in this fixed order with
// no contraction, so h is the same on every IEEE-754 FP64 implementation of
// the same steps.
// ---------------------------------------------------------------------------
template <int D>
__host__ __device__ __forceinline__ void ell_local(const Geom &g, int q, const double *x, double *y) {
#pragma clang fp contract(off)
#pragma unroll
  for (int k = 0; k < D; ++k) {
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < D; ++m) s = s + g.hR[q][3 * k + m] * (x[m] - g.hc[q][m]);
    y[k] = s;
  }
}

template <int D>
__host__ __device__ __forceinline__ double ell_level(const Geom &g, int q, const double *y) {
#pragma clang fp contract(off)
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const double u = y[k] / g.ha[q][k];
    s = s + u * u;
  }
  return s;
}

// Newton step on g(t) = sum_k (a_k y_k / (a_k^2 + t))^2 - 1, whose root t
// gives the closest surface point z_k = a_k^2 y_k / (a_k^2 + t)
template <int D>
__host__ __device__ __forceinline__ double ell_newton(const Geom &g, int q, const double *y, double t) {
#pragma clang fp contract(off)
  double gv = -1.0, dg = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const double a = g.ha[q][k];
    const double e = a * a + t;
    const double u = a * y[k] / e;
    const double uu = u * u;
    gv = gv + uu;
    dg = dg + uu / e;
  }
  return t + gv / (2.0 * dg);
}

// distance to the surface for x outside the hole, 0 inside: g is convex and
// decreasing, and g(t) >= |a y|^2 / (max a^2 + t)^2 - 1, so Newton from
// t0 = max(0, |a y| - max a^2) (left of the root) rises monotonically to it
// and stops when t no longer increases (64 steps at most)
template <int D>
__host__ __device__ __forceinline__ double ell_dist(const Geom &g, int q, const double *x) {
#pragma clang fp contract(off)
  double y[3] = {0.0, 0.0, 0.0};
  ell_local<D>(g, q, x, y);
  if (!(ell_level<D>(g, q, y) > 1.0)) return 0.0;
  double s0 = 0.0, amax2 = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const double a = g.ha[q][k];
    const double ay = a * y[k];
    s0 = s0 + ay * ay;
    amax2 = a * a > amax2 ? a * a : amax2;
  }
  double t = __builtin_sqrt(s0) - amax2;
  t = t > 0.0 ? t : 0.0;
  for (int it = 0; it < 64; ++it) {
    const double tn = ell_newton<D>(g, q, y, t);
    if (!(tn > t)) break;
    t = tn;
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const double a = g.ha[q][k];
    const double z = a * a * y[k] / (a * a + t);
    const double d = y[k] - z;
    s = s + d * d;
  }
  return __builtin_sqrt(s);
}

// closest surface point to a point near the surface: 8 Newton steps from t = 0
template <int D>
__host__ __device__ __forceinline__ void ell_project(const Geom &g, int q, double *x) {
  double y[3] = {0.0, 0.0, 0.0}, z[3] = {0.0, 0.0, 0.0};
  ell_local<D>(g, q, x, y);
  double t = 0.0;
#pragma unroll
  for (int it = 0; it < 8; ++it) t = ell_newton<D>(g, q, y, t);
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const double a = g.ha[q][k];
    z[k] = a * a * y[k] / (a * a + t);
  }
#pragma unroll
  for (int m = 0; m < D; ++m) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) s = s + g.hR[q][3 * k + m] * z[k];
    x[m] = g.hc[q][m] + s;
  }
}

// unit normal of the hole's level set at x, pointing out of the hole
template <int D>
__host__ __device__ __forceinline__ void ell_normal(const Geom &g, int q, const double *x, double *n) {
  double y[3] = {0.0, 0.0, 0.0};
  ell_local<D>(g, q, x, y);
  double gy[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < D; ++k) gy[k] = y[k] / (g.ha[q][k] * g.ha[q][k]);
  double s = 0.0;
#pragma unroll
  for (int m = 0; m < D; ++m) {
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) v = v + g.hR[q][3 * k + m] * gy[k];
    n[m] = v;
    s = s + v * v;
  }
  const double il = 1.0 / __builtin_sqrt(s);
#pragma unroll
  for (int m = 0; m < D; ++m) n[m] *= il;
}

// |x - c_q| in FP32 (for bounds that only prune)
template <int D>
__host__ __device__ __forceinline__ float center_dist32(const Geom &g, int q, const double *p) {
  float s = 0.0f;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const float e = (float)(p[a] - g.hc[q][a]);
    s += e * e;
  }
  return __builtin_sqrtf(s);
}

template <int D>
__host__ __device__ __forceinline__ double h_target(const Geom &g, const double *p) {
#pragma clang fp contract(off)
  if (g.hkind == 0) return g.h0;
  if (g.hkind == 1) {
    double s = 0.0;
    for (int a = 0; a < D; ++a) {
      double d = p[a] - g.hpt[a];
      s = s + d * d;
    }
    return g.h0 + g.grad * __builtin_sqrt(s);
  }
  if (g.hkind == 4) {   // node values of the background grid, multilinear
    int c[3] = {0, 0, 0};
    double t[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < D; ++a) {
      const double top = (double)(g.gn[a] - 1);
      double u = (p[a] - g.glo[a]) * g.gs[a];
      u = u > 0.0 ? u : 0.0;   // also a NaN
      u = u < top ? u : top;
      double f = __builtin_floor(u);
      f = f < top - 1.0 ? f : top - 1.0;
      c[a] = (int)f;
      t[a] = u - f;
    }
    const int nx = g.gn[0], ny = g.gn[1];
    double v[2][2];
    for (int dz = 0; dz < (D == 3 ? 2 : 1); ++dz)
      for (int dy = 0; dy < 2; ++dy) {
        const long long row = ((long long)(c[2] + dz) * ny + (c[1] + dy)) * nx + c[0];
        const double g0 = g.grid[row], g1 = g.grid[row + 1];
        v[dz][dy] = g0 + t[0] * (g1 - g0);
      }
    const double w0 = v[0][0] + t[1] * (v[0][1] - v[0][0]);
    if (D == 2) return w0;
    const double w1 = v[1][0] + t[1] * (v[1][1] - v[1][0]);
    return w0 + t[2] * (w1 - w0);
  }
  if (g.hkind == 3) {   // graded both ways from the sphere |x - point| = dcap
    double s = 0.0;
    for (int a = 0; a < D; ++a) {
      double d = p[a] - g.hpt[a];
      s = s + d * d;
    }
    return g.h0 + g.grad * __builtin_fabs(__builtin_sqrt(s) - g.dcap);
  }
  // |x - c| - min a bounds an ellipsoid's distance from above (its inscribed
  // ball) and |x - c| - max a from below.  An ellipsoid whose lower bound
  // exceeds the smallest upper bound (or the cap) by a relative 1e-12 cannot
  // lower min(d, dcap), so its Newton solve is skipped; the result is the
  // same as with every ellipsoid solved.
  // The bounds only prune, so |x - c| is taken in FP32 (relative error below
  // 1e-6) and widened by a relative 1e-5 in the safe direction.
  double ub = g.dcap;
  for (int q = 0; q < g.nh; ++q) {
    if (!g.hell[q]) continue;
    const double r = (double)center_dist32<D>(g, q, p) * (1.0 + 1e-5);
    double u = r - g.hamin[q];
    u = u > 0.0 ? u : 0.0;
    ub = u < ub ? u : ub;
  }
  double dmin = __builtin_inf();
  for (int q = 0; q < g.nh; ++q) {
    double d;
    if (g.hell[q]) {
      double lim = dmin < g.dcap ? dmin : g.dcap;
      lim = ub < lim ? ub : lim;
      const double r = (double)center_dist32<D>(g, q, p) * (1.0 - 1e-5);
      if (r - g.hamax[q] > lim * (1.0 + 1e-12)) continue;
      d = ell_dist<D>(g, q, p);
    } else {
      double s = 0.0;
      for (int a = 0; a < D; ++a) {
        double e = p[a] - g.hc[q][a];
        s = s + e * e;
      }
      d = __builtin_fabs(__builtin_sqrt(s) - g.hr[q]);
    }
    if (d < dmin) dmin = d;
  }
  if (g.dcap < dmin) dmin = g.dcap;
  return g.h0 * (1.0 + g.grad * dmin);
}

// |x_i - x_j|^2 < c2 max(h_i, h_j)^2 (c2 = (r_c / h)^2) with A4 = c2 (h_a h_a)
// precomputed: c2 max(h_a, h_b)^2 is the larger of c2 h_a^2 and c2 h_b^2
// (squaring and scaling by c2 > 0 are monotone, and both sides round the same
// products), so the predicate holds exactly when s is below either.  The
// squared distance is summed over axes in order, without contraction.
template <int D>
__host__ __device__ __forceinline__ bool within_a4(const double4 &a, double A4, double c2,
                                          const double4 &b) {
#pragma clang fp contract(off)
  double d = a.x - b.x;
  double s = d * d;
  d = a.y - b.y;
  s = s + d * d;
  if (D == 3) {
    d = a.z - b.z;
    s = s + d * d;
  }
  return (s < A4) | (s < c2 * (b.w * b.w));
}

// Workgroups are dispatched round-robin over the 8 XCDs; map them so that
// each XCD (and its L2) works on one contiguous stretch of the cell-ordered
// particles.  gridDim.x is a multiple of 8.
__device__ __forceinline__ int xcd_block() {
#if SPH_XCD_REMAP
  const int per = (int)(gridDim.x >> 3);
  return (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
#else
  return (int)blockIdx.x;
#endif
}

// Lanes of one wave that exchange data through LDS: the writes before this
// point are visible to the reads after it (a wave's LDS operations complete in
// order; the fences keep the compiler from moving them across).
__device__ __forceinline__ void lane_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// the cells of a row (fixed y, z) are consecutive and run along x.  In 3D,
// a level with at least 64 cells along y and z numbers its rows in 8 x 8
// tiles of (y, z): the 64 rows of a tile are consecutive and the tiles
// follow each other row-major.  Rows close in space are then close in the
// cell order, so the particles the sweeps gather from stay in cache.  The
// tiles pad y and z to multiples of 8 (the padding rows hold no particle).
__host__ __device__ __forceinline__ bool rows_tiled(int D, const int *nc) {
  return D == 3 && nc[1] >= 64 && nc[2] >= 64;
}
template <int D>
__host__ __device__ __forceinline__ uint32_t cell_row(const Grid &G, int l, uint32_t cy, uint32_t cz) {
  if (!rows_tiled(D, G.nc[l])) return cz * (uint32_t)G.nc[l][1] + cy;
  const uint32_t nyt = ((uint32_t)G.nc[l][1] + 7u) >> 3;
  return (((cz >> 3) * nyt + (cy >> 3)) << 6) + ((cz & 7u) << 3) + (cy & 7u);
}

__host__ __device__ __forceinline__ int cell_coord(const Grid &G, int l, int a, double p) {
  double t = __builtin_floor((p - G.lo[a]) * G.inv_c[l][a]);
  t = t >= 0.0 ? t : 0.0;   // also maps NaN to cell 0
  double top = (double)(G.nc[l][a] - 1);
  t = t > top ? top : t;
  return (int)t;
}

// cell level of smoothing length h (thresholds ascending; NaN -> level 0)
__host__ __device__ __forceinline__ int h_level(const Grid &G, double h) {
  int l = 0;
  for (int q = 1; q < G.nlev; ++q) l += h >= G.hthr[q] ? 1 : 0;
  return l;
}

// ---------------------------------------------------------------------------
// Wendland C2 kernel at smoothing length h (support 2h) in intrinsic
// dimension k (1, 2, 3):
// W = alpha_k h^-k w(q), w = (1-q/2)^4 (1+2q) (k = 2, 3) or (1-q/2)^3 (1+3q/2)
// (k = 1); (dW/dr)/r = alpha_k h^-(k+2) w'(q)/q with w'(q)/q = -5 (1-q/2)^3 or
// -3 (1-q/2)^2, finite at r = 0.  The intrinsic dimension K is a template
// argument.
// ---------------------------------------------------------------------------
template <int K, typename R>
__host__ __device__ __forceinline__ constexpr R kalphaK() {
  return K == 1 ? R(0.625) : (K == 2 ? R(0.55704230082163367519) : R(0.41778172561622525639));
}
template <int K, typename R>
__host__ __device__ __forceinline__ R wshapeK(R q) {   // w(q), caller guarantees q < 2 or clamps t
  R t = R(1) - R(0.5) * q;
  t = t > R(0) ? t : R(0);
  const R t2 = t * t;
  return K == 1 ? t2 * t * (R(1) + R(1.5) * q) : t2 * t2 * (R(1) + R(2) * q);
}
template <int K, typename R>
__host__ __device__ __forceinline__ R dwqK(R q) {      // w'(q)/q
  R t = R(1) - R(0.5) * q;
  t = t > R(0) ? t : R(0);
  return K == 1 ? R(-3) * t * t : R(-5) * t * t * t;
}
template <int K, typename R>
__host__ __device__ __forceinline__ R powK(R h) {
  return K == 1 ? h : (K == 2 ? h * h : h * h * h);
}

// fast reciprocal / square root per precision
__host__ __device__ __forceinline__ double rcp_(double x) { return 1.0 / x; }
__device__ __forceinline__ float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }
__host__ __device__ __forceinline__ double sqrt_(double x) { return __builtin_sqrt(x); }
__device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }

// Accumulation of pair terms.  Sum<false>: the terms (FP64, or FP32 in the
// FP32-mixed mode) are added in FP64.  Sum<true> (FP32-compensated mode): FP32
// terms added in FP32 with Neumaier's compensation (Neumaier 1974): the
// rounding error of every addition is recovered exactly, from whichever of the
// running sum and the term is larger, and kept in a second FP32 word.
template <bool CMP>
struct Sum;
template <>
struct Sum<false> {
  double s;
  __host__ __device__ __forceinline__ void init(double v) { s = v; }
  template <typename T>
  __host__ __device__ __forceinline__ void add(T v) { s += (double)v; }
  __host__ __device__ __forceinline__ double get() const { return s; }
};
template <>
struct Sum<true> {
  float s, c;
  __device__ __forceinline__ void init(double v) {
    s = (float)v;
    c = 0.0f;
  }
  __device__ __forceinline__ void add(float v) {
    const float t = s + v;
    c += __builtin_fabsf(s) >= __builtin_fabsf(v) ? (s - t) + v : (v - t) + s;
    s = t;
  }
  __device__ __forceinline__ double get() const { return (double)s + (double)c; }
};

// ---------------------------------------------------------------------------
// feature geometry: tangent projection and closest-point projection
// ---------------------------------------------------------------------------
// u <- T_i u: identity on the volume, drop the normal part on a surface, keep
// the tangent part on a curve, zero on a singular point
template <int D>
__host__ __device__ __forceinline__ void tangent(const Geom &g, const Feat &F, const double *x, double *u) {
  switch (F.kind) {
    case K_VOL: return;
    case K_BOXSIDE: u[F.axis] = 0.0; return;
    case K_EDGE3: {
      double keep = u[F.axis];
      u[0] = u[1] = u[2] = 0.0;
      u[F.axis] = keep;
      return;
    }
    case K_HOLE: {
      if (g.hell[F.hole]) {
        double m[3] = {0.0, 0.0, 0.0};
        ell_normal<D>(g, F.hole, x, m);
        if (D == 2) {   // keep the part along the tangent (-n1, n0)
          const double ut = u[0] * (-m[1]) + u[1] * m[0];
          u[0] = ut * (-m[1]);
          u[1] = ut * m[0];
        } else {        // remove the normal part
          const double un = u[0] * m[0] + u[1] * m[1] + u[2] * m[2];
          u[0] -= un * m[0];
          u[1] -= un * m[1];
          u[2] -= un * m[2];
        }
        return;
      }
      const double *c = g.hc[F.hole];
      if (D == 2) {
        double t0 = -(x[1] - c[1]), t1 = x[0] - c[0];
        double il = 1.0 / __builtin_sqrt(t0 * t0 + t1 * t1);
        t0 *= il;
        t1 *= il;
        double ut = u[0] * t0 + u[1] * t1;
        u[0] = ut * t0;
        u[1] = ut * t1;
      } else {
        double m0 = x[0] - c[0], m1 = x[1] - c[1], m2 = x[2] - c[2];
        double il = 1.0 / __builtin_sqrt(m0 * m0 + m1 * m1 + m2 * m2);
        m0 *= il;
        m1 *= il;
        m2 *= il;
        double un = u[0] * m0 + u[1] * m1 + u[2] * m2;
        u[0] -= un * m0;
        u[1] -= un * m1;
        u[2] -= un * m2;
      }
      return;
    }
    case K_POLY: {    // an imported curve: keep the part along the closest segment
      double q[D], t[D];
      seg_tangent<D>(g, poly_closest<D>(g, F.hole, x, q), t);
      if (D == 2) {
        const double ut = u[0] * t[0] + u[1] * t[1];
        u[0] = ut * t[0];
        u[1] = ut * t[1];
        u[2] = 0.0;
      } else {
        const double ut = u[0] * t[0] + u[1] * t[1] + u[2] * t[D - 1];
        u[0] = ut * t[0];
        u[1] = ut * t[1];
        u[2] = ut * t[D - 1];
      }
      return;
    }
    case K_LEVEL: {   // the zero level set: normal from the gradient
      double m[3];
      ls_unit<D>(g, x, m);
      if (D == 2) {
        const double ut = u[0] * (-m[1]) + u[1] * m[0];
        u[0] = ut * (-m[1]);
        u[1] = ut * m[0];
      } else {
        const double un = u[0] * m[0] + u[1] * m[1] + u[2] * m[2];
        u[0] -= un * m[0];
        u[1] -= un * m[1];
        u[2] -= un * m[2];
      }
      return;
    }
    case K_SHELL: {   // the ball domain's sphere: as a ball hole about dc
      const double *c = g.dc;
      if (D == 2) {
        double t0 = -(x[1] - c[1]), t1 = x[0] - c[0];
        double il = 1.0 / __builtin_sqrt(t0 * t0 + t1 * t1);
        t0 *= il;
        t1 *= il;
        double ut = u[0] * t0 + u[1] * t1;
        u[0] = ut * t0;
        u[1] = ut * t1;
      } else {
        double m0 = x[0] - c[0], m1 = x[1] - c[1], m2 = x[2] - c[2];
        double il = 1.0 / __builtin_sqrt(m0 * m0 + m1 * m1 + m2 * m2);
        m0 *= il;
        m1 *= il;
        m2 *= il;
        double un = u[0] * m0 + u[1] * m1 + u[2] * m2;
        u[0] -= un * m0;
        u[1] -= un * m1;
        u[2] -= un * m2;
      }
      return;
    }
    default: u[0] = u[1] = u[2] = 0.0; return;
  }
}

__host__ __device__ __forceinline__ double clamp_(double v, double lo, double hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

// closest point of feature F to x (in place)
template <int D>
__host__ __device__ __forceinline__ void project(const Geom &g, const Feat &F, double *x) {
  switch (F.kind) {
    case K_BOXSIDE:
      for (int a = 0; a < D; ++a) x[a] = clamp_(x[a], g.lo[a], g.hi[a]);
      x[F.axis] = F.side ? g.hi[F.axis] : g.lo[F.axis];
      return;
    case K_EDGE3:
      x[F.axis] = clamp_(x[F.axis], g.lo[F.axis], g.hi[F.axis]);
      x[F.fax0] = F.fsd0 ? g.hi[F.fax0] : g.lo[F.fax0];
      x[F.fax1] = F.fsd1 ? g.hi[F.fax1] : g.lo[F.fax1];
      return;
    case K_HOLE: {
      if (g.hell[F.hole]) {
        ell_project<D>(g, F.hole, x);
        return;
      }
      const double *c = g.hc[F.hole];
      double d[3] = {0.0, 0.0, 0.0}, s = 0.0;
      for (int a = 0; a < D; ++a) {
        d[a] = x[a] - c[a];
        s += d[a] * d[a];
      }
      double r = __builtin_sqrt(s);
      for (int a = 0; a < D; ++a) x[a] = c[a] + g.hr[F.hole] * (d[a] / r);
      return;
    }
    case K_CORNER:
      for (int a = 0; a < D; ++a) x[a] = ((F.bits >> a) & 1) ? g.hi[a] : g.lo[a];
      return;
    case K_POLY: {   // the closest point of the particle's own polyline
      double q[D];
      (void)poly_closest<D>(g, F.hole, x, q);
      for (int a = 0; a < D; ++a) x[a] = q[a];
      return;
    }
    case K_LEVEL:   // 12 Newton steps along the gradient onto phi = 0
      for (int it = 0; it < 12; ++it) {
        double gr[3];
        const double p = ls_phi<D>(g, x, gr);
        double gg = 0.0;
        for (int a = 0; a < D; ++a) gg += gr[a] * gr[a];
        if (!(gg > 0.0)) return;
        for (int a = 0; a < D; ++a) x[a] -= p * gr[a] / gg;
      }
      return;
    case K_SHELL: {
      double d[3] = {0.0, 0.0, 0.0}, s = 0.0;
      for (int a = 0; a < D; ++a) {
        d[a] = x[a] - g.dc[a];
        s += d[a] * d[a];
      }
      double r = __builtin_sqrt(s);
      for (int a = 0; a < D; ++a) x[a] = g.dc[a] + g.dR * (d[a] / r);
      return;
    }
    default: return;
  }
}

// phi(x) > 0: strictly inside the box, strictly outside every hole; or
// strictly inside the ball domain
template <int D>
__host__ __device__ __forceinline__ bool inside(const Geom &g, const double *x) {
#pragma clang fp contract(off)
  if (g.domain == 1) {
    double s = 0.0;
    for (int a = 0; a < D; ++a) {
      double d = x[a] - g.dc[a];
      s = s + d * d;
    }
    return s < g.dR * g.dR;
  }
  if (g.domain == 2) {
    for (int a = 0; a < D; ++a)
      if (!(x[a] > g.lo[a] && x[a] < g.hi[a])) return false;
    double gr[3];
    return ls_phi<D>(g, x, gr) > 0.0;
  }
  for (int a = 0; a < D; ++a)
    if (!(x[a] > g.lo[a] && x[a] < g.hi[a])) return false;
  for (int q = 0; q < g.nh; ++q) {
    double s = 0.0;
    for (int a = 0; a < D; ++a) {
      double d = x[a] - g.hc[q][a];
      s = s + d * d;
    }
    if (g.hell[q]) {
      // beyond the ellipsoid's bounding ball (with a relative 1e-12 to
      // spare) its level exceeds 1 whatever the rounding: no quadric needed
      const double am = g.hamax[q];
      if (s > am * am * (1.0 + 1e-12)) continue;
      double y[3] = {0.0, 0.0, 0.0};
      ell_local<D>(g, q, x, y);
      if (!(ell_level<D>(g, q, y) > 1.0)) return false;
      continue;
    }
    double r = g.hr[q];
    if (!(s > r * r)) return false;
  }
  return true;
}

__device__ __forceinline__ unsigned long long dbits(double v) {
  return (unsigned long long)__double_as_longlong(v);
}
__device__ __forceinline__ double bitsd(unsigned long long b) {
  return __longlong_as_double((long long)b);
}

// ---------------------------------------------------------------------------
// the control law of one feature (sec. 3.4): V-bar sampling every
// sample_every steps into windows of window_samples, E_t against the last
// window mean, E_avg between the last two window means, E_sys = max of both;
// Phase One -> transition when E_sys < tol (or after max_phase1_steps) ->
// Phase Two -> frozen; velocity resets: every reset_period steps and after a
// tenfold time-step drop in Phase One, a halving period in the transition,
// every step in Phase Two.
// ---------------------------------------------------------------------------
__device__ inline void control_law(const Ctl &P, Group &G, double vbar, double dt) {
  G.n_ph += 1;
  if (G.n_ph % P.sample_every == 0) {
    G.vbar = vbar;
    G.ring[G.nring] = vbar;
    G.nring += 1;
    if (G.nring == P.window_samples) {
      double s = 0.0;
      for (int q = 0; q < G.nring; ++q) s = s + G.ring[q];
      G.a_prev = G.a_last;
      G.a_last = s / (double)G.nring;
      G.nwin += 1;
      G.nring = 0;
    }
    double et = G.nwin >= 1 ? __builtin_fabs(vbar - G.a_last) / G.a_last : __builtin_inf();
    double ea = G.nwin >= 2 ? __builtin_fabs(G.a_last - G.a_prev) / G.a_prev : __builtin_inf();
    G.esys = et > ea ? et : ea;
  }
  if (G.phase == PH_ONE) {
    if (G.esys < P.tol || G.n_ph >= P.max_phase1_steps) {
      G.phase = PH_RAMP;
      G.n_ph = 0;
    }
  } else if (G.phase == PH_RAMP) {
    if (G.n_ph >= P.ramp_steps) {
      G.phase = PH_TWO;
      G.n_ph = 0;
    }
  } else if (G.phase == PH_TWO) {
    if (G.n_ph >= P.phase2_steps) G.phase = PH_FROZEN;
  }
  if (G.phase == PH_ONE) {
    G.reset_next = (G.n_ph % P.reset_period == 0) || (G.dt_prev > 0.0 && dt < 0.1 * G.dt_prev);
  } else if (G.phase == PH_RAMP) {
    int shift = G.n_ph / P.ramp_halving;
    int period = shift >= 30 ? 1 : (P.reset_period >> shift);
    if (period < 1) period = 1;
    G.reset_next = (G.n_ph % period) == 0;
  } else {
    G.reset_next = 1;
  }
  G.dt_prev = dt;
}

__device__ inline double damping(const Ctl &P, const Group &G) {
  if (G.phase == PH_ONE) return P.eps_damp;
  if (G.phase == PH_RAMP) return P.eps_damp * (1.0 - (double)G.n_ph / (double)P.ramp_steps);
  return 0.0;
}

}  // namespace sph
