/*
 * sphref.h -- plain FP64 CPU oracle of the feature-aware SPH relaxation step
 * (Ji, Fu, Hu, Adams, "A Feature-aware SPH for Isotropic Unstructured Mesh
 * Generation", arXiv 2003.01061).
 *
 * TEST INFRASTRUCTURE ONLY.  This oracle exists so that the GPU library can be
 * checked against an obviously correct, slow implementation written straight
 * from the paper.  Only the test suite, the smoke check and the benchmark's CPU
 * baseline may load it.  It shares no code, header, table or helper with the
 * GPU library, and it never reads anything the GPU library produced.
 *
 * Everything is double precision, single threaded, compiled without FMA
 * contraction.  Sums run over neighbours in ascending particle id.
 *
 * Particle arrays are row-major n x 3 (unused third coordinate = 0 in 2D) and
 * are indexed by the caller's particle id 0..n-1; the oracle never reorders.
 *
 * Feature numbering (shared convention, implemented independently by each
 * side).  2D box minus discs:
 *   0 volume | 1..4 box edges x=lo, x=hi, y=lo, y=hi | 5..4+nh hole circles |
 *   then 4 corners, corner c at (bit0 ? hi : lo, bit1 ? hi : lo).
 * 3D box minus balls / ellipsoids:
 *   0 volume | 1..6 faces x=lo, x=hi, y=lo, y=hi, z=lo, z=hi |
 *   7..6+nh hole surfaces | 12 box edges | 8 corners.
 *   Edge 4a + sb + 2 sc runs along axis a; its two fixed coordinates are the
 *   other axes b < c, at lo (0) or hi (1) given by sb and sc.
 *   Corner c sits at (bit0, bit1, bit2) ? hi : lo per axis.
 */
#ifndef SPHREF_H
#define SPHREF_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct sphref_job sphref_job;

/* Box [lo,hi]^dim minus n_holes holes.  holes: n_holes x 15 doubles:
 * centre[3], semi_axes[3], rot[9] (row-major, local = rot * (x - centre)).
 * A hole whose semi-axes (the first dim) are equal is a disc (2D) / ball (3D)
 * of that radius and its rotation is ignored; otherwise it is an ellipse /
 * ellipsoid, sum_k (local_k / a_k)^2 <= 1, with an orthonormal rotation. */
typedef struct {
  int32_t dim;
  double lo[3], hi[3];
  int32_t n_holes;
  const double *holes;
  int32_t domain;        /* 0: the box minus the holes; 1: the ball (disc)
                            inscribed in the box, which must be a cube, with
                            no holes: features 0 volume | 1 sphere (circle);
                            2: the positive phase of the level set phi
                            below, within the box, no holes: features
                            0 volume | 1 the zero level set */
  const double *phi;     /* domain 2: phi at the nodes of a Cartesian grid,
                            x fastest, interpolated like the gridded sizing */
  int32_t phi_n[3];
  double phi_lo[3], phi_hi[3];
  /* domain 2 in 2D with imported feature curves (sec. 2.1's sharp edges as
   * polylines, and singular points): curve c has the points
   * curve_pts[3 k], k in [curve_off[c], curve_off[c+1]), runs with the
   * domain on its left, and ends at the corners curve_ends[2c] (its first
   * point) and curve_ends[2c+1] (its last), -1 for none.  Features are then
   * 0 volume | 1..n_curves the curves | then the corners, in order. */
  int32_t n_curves;
  const int32_t *curve_off;
  const double *curve_pts;
  const int32_t *curve_ends;
  int32_t n_corners;
  const double *corners;
  /* domain 2 in 3D with imported curves (sec. 2.1's sharp edges on a 3D
   * level set): the curves split the zero level set into n_patches surface
   * patches; curve c separates patches curve_patches[2c] and
   * curve_patches[2c+1] (0-based, -1 for none).  Features are then
   * 0 volume | 1..n_patches the patches | the curves | the corners.  A
   * curve may be closed (its last point equal to its first, no corners). */
  int32_t n_patches;
  const int32_t *curve_patches;
} sphref_geometry;

/* Target feature size h_t(x) (paper sec. 2.2).
 * kind 0: h = h0
 * kind 1: h = h0 + grad * |x - point|
 * kind 2: h = h0 * (1 + grad * min(d, dcap)), d = distance to the nearest hole
 * kind 3: h = h0 + grad * | |x - point| - dcap |, graded both ways from the
 *         sphere of radius dcap about point
 * kind 4: h sampled at the nodes of a Cartesian grid over [grid_lo, grid_hi]
 *         (grid_n nodes per axis, x fastest), interpolated multilinearly:
 *         per axis s = (n - 1) / (hi - lo), u = (x - lo) s clamped to
 *         [0, n - 1], cell c = min(floor(u), n - 2), t = u - c; then
 *         lerp(a, b, t) = a + t (b - a) along x, then y, then z */
typedef struct {
  int32_t kind;
  double h0, grad, dcap;
  double point[3];
  const double *grid;
  int32_t grid_n[3];
  double grid_lo[3], grid_hi[3];
} sphref_sizing;

typedef struct {
  double p0;               /* EOS constant pressure */
  double eps_damp;         /* Phase One damping factor */
  double tol;              /* E_sys threshold */
  double dt_max;           /* cap when every time-step term is infinite */
  int32_t boundary_weighting; /* 0 rho_t,b*A_t,b = 1/h_b, 1 literal A_t,b, 2 off */
  int32_t reset_period;    /* Phase One velocity reset period */
  int32_t sample_every;    /* steps between V-bar samples */
  int32_t window_samples;  /* samples per time-averaging window */
  int32_t ramp_steps;      /* transition length */
  int32_t ramp_halving;    /* steps between halvings of the reset period */
  int32_t phase2_steps;    /* Phase Two length before a group freezes */
  int32_t max_phase1_steps;/* forced switch out of Phase One */
  int32_t sum_order;       /* neighbour sums: 0 ascending id, 1 descending id
                              (two equally valid rounding orders; their
                              divergence is the noise floor of a trajectory) */
  double kernel_support;   /* cut-off radius r_c in units of h (sec. 2.3 gives
                              no value): the kernel's smoothing length is
                              r_c / 2; 0 = 2 (smoothing length h) */
  double boundary_scale;   /* factor on the boundary term of the pressure
                              force; 0 = 1 (the term as printed; 2 is a
                              mesh-quality calibration that moves the first
                              particle off a boundary to one spacing) */
} sphref_params;

/* fields for sphref_get_field, all from the last completed step */
enum {
  SPHREF_F_H = 0,      /* h_t(x^n)                     n        */
  SPHREF_F_AP = 1,     /* pressure acceleration a^p    n x 3    */
  SPHREF_F_A = 2,      /* total acceleration a         n x 3    */
  SPHREF_F_VT = 3,     /* particle volume V~           n        */
  SPHREF_F_GAMMA = 4,  /* Shepard term gamma           n        */
  SPHREF_F_VMID = 5    /* mid-point velocity v~        n x 3    */
};

/* kernel (Wendland C2 at smoothing length h, support 2h) of intrinsic
 * dimension k = 1, 2, 3 */
double sphref_W(int32_t k, double r, double h);
double sphref_dWdr(int32_t k, double r, double h);
/* target feature size at a point */
double sphref_h_at(const sphref_geometry *g, const sphref_sizing *s, const double *x);
/* closest-point projection of x onto feature f (in place); returns 0 */
int32_t sphref_project(const sphref_geometry *g, int32_t f, double *x);
/* number of features of a geometry and the type (0 SI,1 C,2 S,3 V) of one */
int32_t sphref_n_features(const sphref_geometry *g);
int32_t sphref_feature_type(const sphref_geometry *g, int32_t f);
/* outward normal n_{b|f}: of feature fi's boundary at boundary particle
 * position xb of feature fb; returns 1 if fb bounds fi, 0 otherwise, -1 for
 * a pair whose normal depends on the particle of fi (below) */
int32_t sphref_boundary_normal(const sphref_geometry *g, int32_t fi, int32_t fb,
                               const double *xb, double *n);
/* the same seen from a particle of fi at xi: a 3D surface patch's normal at
 * its curves and corners depends on xi */
int32_t sphref_boundary_normal_at(const sphref_geometry *g, int32_t fi, int32_t fb,
                                  const double *xb, const double *xi, double *n);
/* Tag system of the background grid of a level-set domain (sec. 3.2), one
 * entry per grid cell (cells between the nodes of phi, x fastest):
 *   ctype: 0 negative cell (C-), 1 positive cell (C+), 2 surface cell (C_s),
 *          3 curve cell (C_c), 4 singular cell (C_si)
 *   cindex: the feature index within its type (volume component, surface
 *          patch, curve, corner), -1 for a negative cell.
 * A cell is positive when phi > 0 at all its nodes, negative when phi < 0 at
 * all of them, a surface cell otherwise.  A curve marks the cells its points
 * (sampled at a quarter of the smallest cell side) lie in and their face
 * neighbours; a corner marks its cell and all neighbours; the first curve
 * (corner) in order keeps a cell, corners win over curves.  Surface cells
 * that remain form patches, positive cells volumes: components over face
 * neighbours, numbered in the order of their first cell.  Curve c touches
 * patch p when one of its cells is a face neighbour of a cell of p; the
 * two touched patches go to curve_patches[2c], [2c+1] (ascending, -1 for
 * none; -2 in [2c] if more than two).  Counts go to *n_volumes, *n_patches. */
int32_t sphref_tags(const sphref_geometry *g, int32_t *ctype, int32_t *cindex,
                    int32_t *n_volumes, int32_t *n_patches, int32_t *curve_patches);

int32_t sphref_create(const sphref_geometry *g, const sphref_sizing *s,
                      const sphref_params *p, int64_t n, const double *xyz,
                      const int32_t *feature, sphref_job **out);
void sphref_destroy(sphref_job *j);
int32_t sphref_step(sphref_job *j, int32_t n_steps);
int32_t sphref_set_state(sphref_job *j, const double *xyz, const double *vel);
int32_t sphref_get_state(sphref_job *j, double *xyz, double *vel);
int32_t sphref_get_field(sphref_job *j, int32_t which, double *out);
/* neighbour lists N(i) of the current positions, CSR, ids ascending;
 * rel_out (may be NULL): 1 same group, 2 boundary.  Returns the pair count
 * through n_pairs; fails (-1) when cap is too small (n_pairs still set). */
int32_t sphref_neighbors(sphref_job *j, int64_t *offsets, int32_t *ids,
                         int8_t *rel_out, int64_t cap, int64_t *n_pairs);
/* Sampled check at any size: for the m particles idx[] of the current
 * positions, the neighbour list by brute force over all particles (CSR over
 * the sample, ids ascending) and the sweep-A quantities over it: pressure
 * acceleration a^p (m x 3), particle volume V~ (m), Shepard gamma (m). */
int32_t sphref_sample(sphref_job *j, int32_t m, const int64_t *idx, int64_t *offsets,
                      int32_t *ids, int8_t *rel, int64_t cap, double *ap, double *vt,
                      double *gam);
int32_t sphref_error(sphref_job *j, double *e_sys, int32_t *phase,
                     int32_t *converged, int64_t *step);
/* per-feature control state: out[0..9] = phase, n_phase, E_sys, dt1, dt,
 * last V-bar, reset_next, A_last, A_prev, n_windows */
int32_t sphref_group_state(sphref_job *j, int32_t f, double *out);
/* counters: out[0] steps, out[1] escaped moves, out[2] interactions summed
 * over all steps, out[3] interactions of the last step */
int32_t sphref_counters(sphref_job *j, double *out);
/* Run one group's control law over a synthetic series of per-step V-bar and
 * final time-step values (no particles).  Per step k it writes the phase
 * after the step, whether the velocity is reset at the start of step k+1,
 * and E_sys.  Used to pin the control law by hand-computed cases. */
int32_t sphref_control_replay(const sphref_params *p, int32_t n_steps,
                              const double *vbar, const double *dt,
                              int32_t *phase_out, int32_t *reset_out,
                              double *esys_out);
const char *sphref_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
