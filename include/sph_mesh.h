/*
 * sph_mesh.h -- C ABI of the MI355X (gfx950) feature-aware SPH relaxation
 * library libsphmesh.so.
 *
 * The library runs the per-step particle relaxation of Ji, Fu, Hu and Adams,
 * "A Feature-aware SPH for Isotropic Unstructured Mesh Generation" (arXiv
 * 2003.01061), Algorithm 1's time loop, entirely in hand-written HIP kernels:
 * cell hashing and counting sort, cell start tables, the neighbour-list sweep,
 * the Shepard / pressure / boundary-correction force sweep, the viscous sweep,
 * integration with feature projection, and the per-feature time step, error
 * measure and two-phase control.  The host only enqueues work.
 *
 * Conventions for every call:
 *  - Every pointer argument is a HOST pointer unless stated otherwise.
 *    Inputs are copied during the call; the caller keeps ownership.
 *  - Outputs go to caller-owned host buffers.
 *  - Calls return an sph_status; on failure sph_mesh_last_error() returns a
 *    message (thread-local, valid until the next call on that thread).
 *  - One handle must not be used from two threads at once; distinct handles
 *    are independent (each owns its device memory and stream).
 *  - Particle arrays are row-major n x 3 doubles (the third coordinate is
 *    ignored in 2D) indexed by the caller's particle id 0..n-1.  The library
 *    keeps particles in cell order internally and always reports in the
 *    caller's order.
 *
 * Feature numbering (a feature is the paper's (type, index) pair, sec. 3.2;
 * each feature evolves as one group with its own time step, sec. 3.5):
 *   2D box [lo,hi]^2 minus n_holes discs / ellipses:
 *     0 volume (P_+) | 1..4 box edges x=lo, x=hi, y=lo, y=hi (P_c) |
 *     5..4+n_holes hole boundaries (P_c) | then 4 corners (P_si), corner c at
 *     (bit0 of c ? hi : lo, bit1 of c ? hi : lo).
 *   3D box [lo,hi]^3 minus n_holes balls / ellipsoids:
 *     0 volume (P_+) | 1..6 faces x=lo, x=hi, y=lo, y=hi, z=lo, z=hi (P_s) |
 *     7..6+n_holes hole surfaces (P_s) | 12 box edges (P_c) | 8 corners (P_si).
 *     Edge 4a + sb + 2 sc runs along axis a; its fixed coordinates are the
 *     two other axes b < c, at lo (0) or hi (1) as given by sb and sc.
 *     Corner c sits at (bit0, bit1, bit2 of c) ? hi : lo per axis.
 */
#ifndef SPH_MESH_H
#define SPH_MESH_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sph_mesh sph_mesh;

typedef enum {
  SPH_OK = 0,
  SPH_ERR_INVALID_ARG = 1,   /* bad geometry, sizing, parameters or buffer */
  SPH_ERR_OUT_OF_MEMORY = 2, /* device allocation failed, or a batch is full */
  SPH_ERR_DEVICE = 3,        /* a HIP call failed */
  SPH_ERR_STATE = 4,         /* non-finite state or neighbour-list overflow */
  SPH_ERR_UNSUPPORTED = 5    /* a configuration this build does not handle */
} sph_status;

enum { SPH_P_SINGULAR = 0, SPH_P_CURVE = 1, SPH_P_SURFACE = 2, SPH_P_VOLUME = 3 };
enum { SPH_H_CONST = 0, SPH_H_LINEAR_FROM_POINT = 1, SPH_H_GRADED_TO_HOLES = 2, SPH_H_SHELL = 3,
       SPH_H_GRID = 4 };
enum { SPH_DOMAIN_BOX = 0, SPH_DOMAIN_BALL = 1, SPH_DOMAIN_LEVEL_SET = 2 };
enum { SPH_FP64 = 0, SPH_FP32_MIXED = 1, SPH_FP32_COMPENSATED = 2 };

/* Geometry (paper sec. 2.1 / 3.1): the level set phi > 0 is the box minus
 * the holes.  holes: n_holes x 15 doubles, centre[3], semi_axes[3], rot[9]
 * (row-major, orthonormal): the hole is sum_k (y_k / a_k)^2 <= 1 with local
 * coordinates y = rot (x - centre) (the first dim axes).  Equal semi-axes
 * make a disc / ball (rot ignored; closed-form projections); otherwise an
 * ellipse / ellipsoid, whose closest points come from Newton's method on
 * the Lagrange multiplier t of z_k = a_k^2 y_k / (a_k^2 + t) (8 fixed steps
 * to project a particle, until t stops increasing for the distance in h_t).
 * At most 16 holes; each must lie inside the box with a margin of its
 * largest semi-axis; every particle must lie in the box. */
typedef struct {
  int32_t dim;               /* 2 or 3 */
  double lo[3], hi[3];
  int32_t n_holes;
  const double *holes;
  int32_t domain;            /* SPH_DOMAIN_BOX (0): the box minus the holes,
                                features as numbered above.
                                SPH_DOMAIN_BALL (1): the ball (disc) inscribed
                                in the box, as for sec. 4's sphere cases; the
                                box must be a cube and there are no holes;
                                features 0 volume, 1 its sphere (circle).
                                SPH_DOMAIN_LEVEL_SET (2): the positive phase
                                of the level set phi below, within the box,
                                no holes (sec. 2.1); features 0 volume phi > 0,
                                1 the zero level set.  A particle of feature 1
                                is mapped onto phi = 0 by 12 Newton steps
                                x <- x - phi grad / |grad|^2; the normal out of
                                the domain is -grad / |grad| */
  const double *phi;         /* SPH_DOMAIN_LEVEL_SET: phi at the nodes of a
                                Cartesian grid (host memory, copied by the
                                library), laid out and interpolated as the
                                gridded sizing's values; grad is the
                                derivative of that multilinear function in
                                the cell of x */
  int32_t phi_n[3];
  double phi_lo[3], phi_hi[3];
  /* SPH_DOMAIN_LEVEL_SET may import sharp features (sec. 2.1): feature
   * curves as polylines and singular points.  Curve c has the points
   * curve_pts[3 k .. 3 k + 2], k in [curve_off[c], curve_off[c + 1]) (at
   * least 2, consecutive points distinct), in 2D runs with the domain on its
   * left, and ends at the corners curve_ends[2 c] (first point) and
   * curve_ends[2 c + 1] (last point), -1 for none; corners[3 m ..] is corner
   * m.  A curve particle is mapped to the closest point of its own polyline
   * (the first segment on ties) and moves along that segment; a curve's
   * normal at its end corner runs along its end segment, away from the
   * curve.  n_curves = 0: no imported features.  All arrays are host memory,
   * copied by the library.
   * 2D: features 0 volume | 1 .. n_curves the curves | the corners (no
   * zero-level-set feature); the volume's normal at a curve particle is the
   * segment's right normal; at a corner, the normalised sum of the right
   * normals of the end segments meeting there.  n_patches must be 0.
   * 3D: the curves split the zero set into n_patches >= 1 surface patches
   * (sph_tags finds them); curve c lies between patches curve_patches[2 c]
   * and curve_patches[2 c + 1] (-1 for none).  Features: 0 volume |
   * 1 .. n_patches the patches | the curves | the corners.  A patch particle
   * is mapped onto phi = 0 as above; a patch is bounded by the curves beside
   * it and their end corners, with the normal
   * (I - t t^T)(I - m m^T)(x_b - x_i), normalised (m the patch's unit normal
   * at the particle x_i, t the unit tangent of b's closest segment; at a
   * corner without the t part); the volume's normal at a curve or corner
   * particle is -grad / |grad| of phi there. */
  int32_t n_curves;
  const int32_t *curve_off;
  const double *curve_pts;
  const int32_t *curve_ends;
  int32_t n_corners;
  const double *corners;
  int32_t n_patches;
  const int32_t *curve_patches;
} sph_geometry;

/* Target feature size h_t(x) (paper sec. 2.2):
 *   SPH_H_CONST:             h = h0
 *   SPH_H_LINEAR_FROM_POINT: h = h0 + grad |x - point|
 *   SPH_H_GRADED_TO_HOLES:   h = h0 (1 + grad min(d, dcap)), d = distance to
 *                            the nearest hole boundary.
 *   SPH_H_SHELL:             h = h0 + grad | |x - point| - dcap |, graded both
 *                            ways from the sphere of radius dcap about point
 *                            (sec. 4's Sphere02).
 *   SPH_H_GRID:              h sampled at the nodes of a Cartesian background
 *                            grid (sec. 2.2 keeps h_t on the background
 *                            mesh): grid_n[a] nodes on axis a over
 *                            [grid_lo[a], grid_hi[a]] (grid_n[2] = 1 in 2D),
 *                            values x fastest, index (k ny + j) nx + i, all
 *                            finite and positive.  Interpolated
 *                            multilinearly: per axis s = (n - 1) /
 *                            (hi - lo), u = (x - lo) s clamped to [0, n - 1],
 *                            c = min(floor(u), n - 2), t = u - c; then
 *                            a + t (b - a) along x, then y, then z.  The
 *                            library copies the grid; the caller's array is
 *                            only read during the call that adds the job.
 * Evaluated in FP64 with the operation order: squared distances summed over
 * axes in order, then sqrt; no fused multiply-add. */
typedef struct {
  int32_t kind;
  double h0, grad, dcap;
  double point[3];
  const double *grid;        /* SPH_H_GRID: node values (host memory) */
  int32_t grid_n[3];
  double grid_lo[3], grid_hi[3];
} sph_sizing;

/* Simulation parameters (paper sec. 2.3, 3.4, 3.5). */
typedef struct {
  double p0;                 /* EOS constant pressure P0 (sec. 2.3) */
  double eps_damp;           /* Phase One damping factor, [0, 0.2] (sec. 3.4.3) */
  double tol;                /* E_sys threshold, 5e-6 in the paper (sec. 3.4.2) */
  double dt_max;             /* time-step cap when every term is infinite */
  int32_t boundary_weighting;/* boundary term weight: 0 rho_t,b A_t,b = 1/h_b,
                                1 the literal A_t,b = h_b^(k-1), 2 off */
  int32_t reset_period;      /* Phase One velocity reset period (100) */
  int32_t sample_every;      /* V-bar sampling interval (20) */
  int32_t window_samples;    /* samples per averaging window (10), <= 64 */
  int32_t ramp_steps;        /* transition length between the phases (140) */
  int32_t ramp_halving;      /* steps between halvings of the reset period (20) */
  int32_t phase2_steps;      /* Phase Two length before a feature freezes (400) */
  int32_t max_phase1_steps;  /* forced end of Phase One */
  int32_t precision;         /* SPH_FP64: every step in FP64.
                                SPH_FP32_MIXED: kernel evaluations and pair
                                terms in FP32, their sums accumulated in FP64;
                                FP64 positions, integration and projection
                                (the viscous pair terms take neighbour
                                positions and h from their FP32 records; the
                                per-particle division by gamma, 1 / S and the
                                time-step terms use FP32 reciprocals and roots).
                                SPH_FP32_COMPENSATED: as SPH_FP32_MIXED with
                                the sums in FP32 too, each with Neumaier
                                compensation */
  int32_t max_neighbors;     /* neighbour-list capacity per particle, rounded up
                                to a multiple of 8; 0 = 104 in 2D, 320 in 3D */
  double cell_factor;        /* cell side = r_c,min cell_factor, r_c,min the
                                support radius kernel_support h_min (0 = 1.0), enlarged
                                if the grid would exceed 2^29 cells */
  int32_t scan_tile;         /* candidate records tested per pass of the
                                neighbour scan: 2, 4 or 8; 0 = 4.  Results do
                                not depend on it (autotuning knob) */
  int32_t cell_levels;       /* cell grids per band of h: level l holds the
                                particles with h_min 2^l <= h < h_min 2^(l+1)
                                on cells of side kernel_support h_min 2^l
                                cell_factor.
                                0 = one level per factor 2 when h_max > 4 h_min
                                (else 1), 1 = a single grid, k <= 6 = at most
                                k levels.  Lists do not depend on it */
  double kernel_support;     /* cut-off radius r_c in units of h (sec. 2.3 names
                                r_c without a value):
                                the kernel is Wendland C2 at smoothing length
                                r_c / 2, neighbours satisfy |x_i - x_j| <
                                r_c max(h_i, h_j) / h, and r_c enters the time
                                step and the viscosity.  0 = 2 (smoothing
                                length h); [1, 8].  2.5 is a mesh-quality
                                calibration (more regular triangles on the
                                paper's square) */
  double boundary_scale;     /* factor on the boundary term of the pressure
                                force (sec. 3.3).  0 = 1, the term as printed:
                                it balances the truncated interior sum
                                exactly, leaving the first particle half a
                                spacing off a boundary.  2 is a mesh-quality
                                calibration that places it one spacing off;
                                [0.25, 8] */
  int32_t use_graph;         /* 1: steps replay captured HIP graphs (of 16
                                and 2 steps) */
  int32_t debug_fields;      /* 1: keep gamma, V~ and v~ for sph_mesh_field */
  void *stream;              /* hipStream_t to run on (e.g. PyTorch's current
                                stream), default priority; NULL = the library
                                creates its own */
  /* Problem statement of sph_mesh_create (Algorithm 1's set-up; ignored by
   * the calls that take the caller's particles): */
  int64_t n_particles;       /* particle budget, split over the features by
                                their masses (sec. 3.2) with h scaled to fit
                                it (reading R25); 0 = the masses as they are */
  uint64_t seed;             /* seed of the 64-bit Mersenne Twister of the
                                initial sampling (sec. 3.6) */
  int32_t init;              /* SPH_INIT_DENSITY: positions drawn with
                                probability proportional to rho_t (sec. 3.6);
                                SPH_INIT_UNIFORM: uniform on each feature */
  int32_t mass_res;          /* points per axis of the mass quadrature; 0 =
                                1024 in 2D, 128 in 3D */
  /* Device memory: dev_alloc(bytes, alloc_ctx) returns device memory (or
   * NULL), dev_free(ptr, alloc_ctx) releases it; for instance PyTorch's
   * caching allocator.  Both NULL = hipMalloc / hipFree.  The library frees
   * only after its stream has drained. */
  void *(*dev_alloc)(size_t bytes, void *ctx);
  void (*dev_free)(void *ptr, void *ctx);
  void *alloc_ctx;
  double verlet_skin;        /* Algorithm 1's Verlet neighbour list as a
                                candidate list of reach (r_c / h + skin) h,
                                built with a re-sort of the particles only when
                                some particle has moved farther than the skin
                                allows since the last build (decided on the
                                device), and filtered into the neighbour list
                                every step; the lists stay those of the cut-off
                                radius.  0 = no candidate list (a cell scan and
                                a sort every step); [0, 2] */
} sph_params;

enum { SPH_INIT_DENSITY = 0, SPH_INIT_UNIFORM = 1 };

/* sph_mesh_create -- Algorithm 1's set-up from the problem statement: the
 * geometry (sec. 2.1), the target feature size h_t (sec. 2.2) and the
 * simulation parameters.  The host integrates rho_t = h^-k over every
 * feature (sec. 3.2's masses M_k; midpoint sums on params->mass_res points per
 * axis), splits params->n_particles over the features at unit mass with h
 * scaled by the s that makes sum_k M_k / s^k equal the budget (h0 and the
 * slope of the linear and two-way sizings multiply by s), places one fixed
 * particle on every box corner, and draws the others from a 64-bit Mersenne
 * Twister seeded with params->seed, with probability proportional to rho_t
 * (params->init = SPH_INIT_DENSITY, sec. 3.6) or uniformly
 * (SPH_INIT_UNIFORM); then it creates the job as
 * sph_mesh_create_with_particles does.  sph_mesh_setup_info reports s and
 * the counts.  Box and ball domains with the analytic sizings;
 * SPH_ERR_UNSUPPORTED for a level-set domain or a gridded sizing (give their
 * particles to sph_mesh_create_with_particles).  Errors as below; *out is
 * NULL on failure. */
sph_status sph_mesh_create(const sph_geometry *geometry, const sph_sizing *sizing,
                           const sph_params *params, sph_mesh **out);

/* sph_mesh_setup_info -- for a job made by sph_mesh_create: the factor h_t
 * was scaled by and the particles placed on every feature (counts[f], cap =
 * capacity of counts; *n_features receives the feature count).  Any output
 * may be NULL; a job made from the caller's particles reports s = 1 and no
 * features. */
sph_status sph_mesh_setup_info(sph_mesh *m, double *h_scale, int64_t *counts, int32_t cap,
                               int32_t *n_features);

/* sph_job_setup -- the host part of sph_mesh_create alone, with no GPU
 * call: *h_scale = s, the scaled h0 and slope (*h0_scaled, *grad_scaled:
 * the sizing the job runs with), the particles per feature (counts[f],
 * counts_cap its capacity, *n_features the feature count) and, when xyz or
 * feature is not NULL, the initial particles themselves (xyz: n x 3 host
 * doubles, feature: n int32, capacity = their particle capacity; *n_out = n),
 * for instance to add the job to a batch with sph_batch_add.  Any output may
 * be NULL.  Errors as sph_mesh_create, and SPH_ERR_INVALID_ARG for a capacity
 * below the counts. */
sph_status sph_job_setup(const sph_geometry *geometry, const sph_sizing *sizing,
                         const sph_params *params, double *h_scale, double *h0_scaled,
                         double *grad_scaled, int64_t *counts, int32_t counts_cap,
                         int32_t *n_features, double *xyz, int32_t *feature, int64_t capacity,
                         int64_t *n_out);

/* sph_tags -- the tag system of a level-set domain's background grid
 * (sec. 3.2), host only (no GPU call).  The cells lie between the nodes of
 * phi, (phi_n[0] - 1) x (phi_n[1] - 1) x (phi_n[2] - 1 in 3D, else 1), x
 * fastest; ctype and cindex (caller-owned host arrays of that many int32)
 * receive per cell:
 *   ctype  0 negative (C-), 1 positive (C+), 2 surface (C_s), 3 curve (C_c),
 *          4 singular (C_si);
 *   cindex the index within its type (volume, patch, curve, corner), -1 for
 *          a negative cell.
 * A cell is positive when phi > 0 at all its nodes, negative when phi < 0 at
 * all of them, surface otherwise.  A curve marks the cells of points along
 * each segment (ceil(length / (s / 4)) steps, s the smallest cell side, both
 * ends included) and their face neighbours; a corner its cell and all its
 * neighbours.  The first curve (corner) in order keeps a cell; corners win
 * over curves.  The remaining surface cells form patches, the positive cells
 * volumes: components under face adjacency, numbered in the order of their
 * first cell.  curve_patches[2 c], [2 c + 1] (2 n_curves int32, may be NULL
 * when n_curves = 0) receive the patches with a cell face-adjacent to a cell
 * of curve c, ascending, -1 for none, -2 in [2 c] for more than two; *n_volumes
 * and *n_patches the counts.  In 3D the geometry's own n_patches and
 * curve_patches may be unset (0 / NULL): the result is how to set them.
 * Errors: SPH_ERR_INVALID_ARG for a bad geometry, a domain other than
 * SPH_DOMAIN_LEVEL_SET or a NULL output. */
sph_status sph_tags(const sph_geometry *geometry, int32_t *ctype, int32_t *cindex,
                    int32_t *n_volumes, int32_t *n_patches, int32_t *curve_patches);

/* sph_mesh_create_with_particles -- the same set-up with the caller's
 * initial particles: n particles at xyz (n x 3) with feature index
 * feature[i] (numbering above; the feature fixes the particle type P_si /
 * P_c / P_s / P_+, sec. 3.2).  Copies everything to the device, builds the
 * feature tables and the cell grid, and returns a handle in *out
 * (library-owned until destroy).  Errors: SPH_ERR_INVALID_ARG for a bad
 * description or a feature index out of range, SPH_ERR_OUT_OF_MEMORY,
 * SPH_ERR_DEVICE.  *out is NULL on failure. */
sph_status sph_mesh_create_with_particles(const sph_geometry *geometry, const sph_sizing *sizing,
                                          const sph_params *params, int64_t n, const double *xyz,
                                          const int32_t *feature, sph_mesh **out);

/* sph_mesh_step -- enqueue n_steps relaxation steps (Algorithm 1's loop body
 * for every feature that has not converged, all features read x^n) on the
 * handle's stream and return without waiting.  A step on a converged job does
 * no work.  Errors that happen on the device are reported by the next
 * positions / error call. */
sph_status sph_mesh_step(sph_mesh *m, int32_t n_steps);

/* sph_mesh_positions -- wait for the stream and copy positions (n x 3, caller
 * order) and, if feature is not NULL, each particle's feature.  With xyz ==
 * NULL only *n_out is set (size query).  capacity is the particle capacity of
 * the buffers.  SPH_ERR_STATE if a non-finite position or a list overflow
 * occurred. */
sph_status sph_mesh_positions(sph_mesh *m, double *xyz, int32_t *feature,
                              int64_t capacity, int64_t *n_out);

/* sph_mesh_error -- wait for the stream; report the convergence error E_sys
 * of sec. 3.4.2 (maximum over moving features; +inf until two averaging
 * windows exist), the least advanced phase (1 Phase One, 2 transition,
 * 3 Phase Two, 4 converged), whether every feature has converged, and the
 * number of steps run.  Any output pointer may be NULL. */
sph_status sph_mesh_error(sph_mesh *m, double *e_sys, int32_t *phase,
                          int32_t *converged, int64_t *step);

/* sph_mesh_destroy -- wait for the stream, free everything; NULL-safe. */
void sph_mesh_destroy(sph_mesh *m);

/* sph_mesh_last_error -- message of the last failure on this thread. */
const char *sph_mesh_last_error(void);

/* ---- inspection and test entry points --------------------------------- */

/* Replace positions (n x 3) and/or velocities (n x 3), caller order; either
 * may be NULL.  Waits for the stream. */
sph_status sph_mesh_set_state(sph_mesh *m, const double *xyz, const double *vel);

/* Copy velocities (n x 3, caller order) after waiting for the stream. */
sph_status sph_mesh_velocities(sph_mesh *m, double *vel);

/* Neighbour lists N(i) of the current positions (Algorithm 1's "construct
 * Verlet neighbor list"): j != i with |x_i - x_j|^2 < c^2 max(h_i, h_j)^2,
 * c = kernel_support
 * (FP64, squared distance summed over axes in order, no fused operations)
 * and an interaction between the features (same feature: rel 1; j on the
 * boundary of i's feature and of lower dimension: rel 2).  CSR in caller
 * order: offsets[n+1], ids ascending per particle, rel per entry (NULL
 * allowed).  Singular particles have empty lists.  With ids == NULL only
 * offsets and *n_pairs are written.  cap = capacity of ids / rel. */
sph_status sph_mesh_neighbors(sph_mesh *m, int64_t *offsets, int32_t *ids,
                              int8_t *rel, int64_t cap, int64_t *n_pairs);

/* Neighbour lists of the count particles idx[0..count) (caller ids) at the
 * current positions, as sph_mesh_neighbors writes them but for those
 * particles only: offsets[count+1], ids / rel per entry (NULL allowed).
 * Copies only the requested lists to the host, so it suits jobs whose whole
 * list set is too large to pull.  SPH_ERR_INVALID_ARG for an index outside
 * [0, n) or cap below the pair count. */
sph_status sph_mesh_neighbors_of(sph_mesh *m, int32_t count, const int64_t *idx,
                                 int64_t *offsets, int32_t *ids, int8_t *rel, int64_t cap,
                                 int64_t *n_pairs);

/* Per-particle quantities of the last step, caller order (needs
 * debug_fields for 3..5): 0 h (n), 1 pressure acceleration a^p (n x 3),
 * 2 acceleration a (n x 3), 3 particle volume V~ (n), 4 Shepard gamma (n),
 * 5 mid-point velocity v~ (n x 3). */
sph_status sph_mesh_field(sph_mesh *m, int32_t which, double *out);

/* Control state of one feature: out[0..9] = phase, steps in phase, E_sys,
 * first time step, final time step, last V-bar sample, velocity reset due at
 * the next step, last window mean, previous window mean, windows seen. */
sph_status sph_mesh_group_state(sph_mesh *m, int32_t feature, double *out);

/* Counters: out[0] steps, out[1] rejected volume-particle moves, out[2]
 * interactions (neighbour-list entries of moving particles) summed over all
 * steps, out[3] interactions of the last step. */
sph_status sph_mesh_counters(sph_mesh *m, double *out);

/* Verlet candidate lists built since creation (each build also re-sorts the
 * particles), for a job created with verlet_skin > 0; 0 otherwise.  Waits
 * for the stream. */
sph_status sph_mesh_list_builds(sph_mesh *m, int64_t *builds);

/* Run the device control law of one feature over a synthetic series of
 * per-step V-bar samples and final time steps (no particles), writing per
 * step the phase after it, whether the velocity is reset at the next step,
 * and E_sys.  n <= 1,000,000. */
sph_status sph_mesh_control_replay(const sph_params *params, int32_t n,
                                   const double *vbar, const double *dt,
                                   int32_t *phase, int32_t *reset, double *e_sys);

/* sph_mesh_control_replay without any allocation, for callers that cannot
 * allocate (code under HIP graph capture, serving loops that must not call
 * hipMalloc).  Same law and results as sph_mesh_control_replay, but vbar, dt
 * (n doubles each), phase, reset (n int32 each) and e_sys (n doubles) are
 * DEVICE pointers owned by the caller, and the work is enqueued on stream
 * (a hipStream_t; NULL = the null stream) without waiting: the outputs are
 * ready when the stream reaches this point.  n <= 1,000,000 (larger series:
 * SPH_ERR_INVALID_ARG).  The only scratch is one feature's control state in
 * a fixed device array of the library (about 700 bytes per GPU, kept until
 * the process ends), re-initialised by every call; calls that overlap on one
 * GPU (other streams, other threads) race on it and must be serialised by
 * the caller.  Errors: SPH_ERR_INVALID_ARG, SPH_ERR_DEVICE (launch failure). */
sph_status sph_mesh_control_replay_noalloc(const sph_params *params, int32_t n,
                                           const double *vbar, const double *dt,
                                           int32_t *phase, int32_t *reset, double *e_sys,
                                           void *stream);

/* Kernel timing with HIP events on the handle's stream.  enable != 0 makes
 * later steps launch without a graph and bracket every kernel with events;
 * sph_mesh_kernel_stats waits for the stream and returns, for kernel `kid`
 * (see sph_mesh_kernel_name), the summed duration in ms and the launch count
 * since profiling was enabled.  Kernel ids are 0..sph_mesh_kernel_count()-1. */
sph_status sph_mesh_profile(sph_mesh *m, int32_t enable);
sph_status sph_mesh_kernel_stats(sph_mesh *m, int32_t kid, double *ms, int64_t *launches);
int32_t sph_mesh_kernel_count(void);
const char *sph_mesh_kernel_name(int32_t kid);

/* Wait for the handle's stream. */
sph_status sph_mesh_sync(sph_mesh *m);

/* ---- batches: many jobs advanced by the same launches ------------------ */
/* A batch keeps several jobs resident on one GPU and advances all of them
 * with one sequence of kernel launches per step (one captured graph), so
 * small jobs share the launch cost.  Every job keeps its own geometry,
 * sizing, parameters, time steps and control state (sec. 3.4-3.5 per job);
 * jobs never interact, and a job's result is bit-identical alone or in any
 * mix.  Jobs can be added and removed between steps (continuous batching).
 * The sph_mesh_* calls above are a batch holding one job. */
typedef struct sph_batch sph_batch;

typedef struct {
  int32_t dim;               /* 2 or 3, shared by every job of the batch */
  int32_t precision;         /* SPH_FP64, SPH_FP32_MIXED or SPH_FP32_COMPENSATED,
                                shared */
  int64_t max_particles;     /* capacity: particles of all resident jobs */
  int64_t max_cells;         /* capacity: cells of all resident jobs' grids */
  int32_t max_jobs;          /* resident jobs, 1..64 */
  int32_t max_neighbors;     /* 0 = 104 in 2D, 320 in 3D */
  int32_t scan_tile;         /* 2, 4 or 8 (0 = 4), as in sph_params */
  int32_t use_graph;         /* 1: steps replay captured graphs of 16 and 2
                                steps (captured on the first multi-step call) */
  int32_t debug_fields;      /* keep gamma, V~, v~ (single-job inspection) */
  void *stream;              /* hipStream_t; NULL = the batch creates its own */
  void *(*dev_alloc)(size_t bytes, void *ctx);   /* as in sph_params; both NULL = */
  void (*dev_free)(void *ptr, void *ctx);        /* hipMalloc / hipFree       */
  void *alloc_ctx;
  double verlet_skin;        /* as in sph_params, for every job of the batch
                                (the jobs' own values are not used); the
                                candidate lists hold up to max_neighbors
                                ((2 + skin) / 2)^dim entries per particle */
} sph_batch_params;

/* Device bytes a batch with these capacities allocates (admission control);
 * -1 on invalid parameters. */
int64_t sph_batch_footprint(const sph_batch_params *bp);

/* Cells of the grid a job would use in a batch (its cell_factor and sizing),
 * or -1 if the description is invalid. */
int64_t sph_job_cells(const sph_geometry *geometry, const sph_sizing *sizing,
                      const sph_params *params);

/* Allocate an empty batch.  SPH_ERR_OUT_OF_MEMORY if the capacities do not
 * fit; *out is NULL on failure. */
sph_status sph_batch_create(const sph_batch_params *bp, sph_batch **out);

/* Add a job (same arguments as sph_mesh_create_with_particles; the batch's dimension,
 * precision, neighbour capacity, graph, debug and stream settings apply, the
 * job's own ones are ignored).  Waits for the stream.  *job receives the
 * job's slot id.  SPH_ERR_OUT_OF_MEMORY when the batch has no room for its
 * particles, cells or slot (the batch is unchanged). */
sph_status sph_batch_add(sph_batch *b, const sph_geometry *geometry, const sph_sizing *sizing,
                         const sph_params *params, int64_t n, const double *xyz,
                         const int32_t *feature, int32_t *job);

/* Remove a job and compact the others.  Waits for the stream. */
sph_status sph_batch_remove(sph_batch *b, int32_t job);

/* Enqueue n_steps steps of every resident job that has not converged. */
sph_status sph_batch_step(sph_batch *b, int32_t n_steps);

/* One synchronisation, then per job slot 0..cap-1: resident (live), converged,
 * and steps run.  Any output may be NULL. */
sph_status sph_batch_status(sph_batch *b, int32_t *live, int32_t *converged, int64_t *steps,
                            int32_t cap);

/* Per-job results (same meaning as the sph_mesh_* calls). */
sph_status sph_batch_positions(sph_batch *b, int32_t job, double *xyz, int32_t *feature,
                               int64_t capacity, int64_t *n_out);
sph_status sph_batch_error(sph_batch *b, int32_t job, double *e_sys, int32_t *phase,
                           int32_t *converged, int64_t *step);
sph_status sph_batch_counters(sph_batch *b, int32_t job, double *out);

/* Verlet candidate lists the batch has built (all its jobs at once), as
 * sph_mesh_list_builds. */
sph_status sph_batch_list_builds(sph_batch *b, int64_t *builds);

/* Wait until every step enqueued on the batch's stream has finished. */
sph_status sph_batch_sync(sph_batch *b);

/* Wait for the batch's stream, free everything; NULL-safe. */
void sph_batch_destroy(sph_batch *b);

/* Device bytes held by the handle. */
int64_t sph_mesh_device_bytes(sph_mesh *m);

#ifdef __cplusplus
}
#endif
#endif
