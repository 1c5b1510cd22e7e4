// sph_mesh.hip -- host runtime and C ABI of libsphmesh.so (include/sph_mesh.h).
//
// One handle = one relaxation job: device-resident particle columns (double
// buffered for the per-step counting sort), the cell grid, the ELL neighbour
// list, the per-feature group table and a status block.  sph_mesh_step only
// enqueues kernels (optionally as a replayed HIP graph of two steps, so the
// double-buffer parity is the same at every replay); control decisions are
// taken on the device, and the host reads state back only when asked.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/sph_mesh.h"
#include "sph_kernels.h"

using namespace sph;

namespace {

thread_local std::string g_err;

sph_status fail(sph_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
sph_status fail(sph_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIPCHK(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(SPH_ERR_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_));      \
  } while (0)

enum KernelId {
  KID_SCAN = 0, KID_SCATTER, KID_RANK_GATHER, KID_NBR_FORCES, KID_REDUCE_A, KID_SWEEP_B,
  KID_REDUCE_B, KID_INTEGRATE_HASH, KID_CONTROL, KID_HASH, KID_NBR_LISTS, KID_COUNT
};
const char *kKernelNames[KID_COUNT] = {
    "scan", "scatter", "rank_gather", "nbr_forces", "reduce_a", "sweep_b", "reduce_b",
    "integrate_hash", "control", "hash", "nbr_lists"};

// ---------------------------------------------------------------------------
// features of a box-minus-holes geometry (numbering of sph_mesh.h)
// ---------------------------------------------------------------------------
struct HFeat {
  int type, k, kind, axis = 0, side = 0, fax[2] = {0, 0}, fsd[2] = {0, 0}, hole = 0, bits = 0;
};

std::vector<HFeat> make_features(int D, int nh) {
  std::vector<HFeat> F;
  F.push_back({T_V, D, K_VOL});
  for (int a = 0; a < D; ++a)
    for (int s = 0; s < 2; ++s) {
      HFeat f{D == 2 ? T_C : T_S, D - 1, K_BOXSIDE};
      f.axis = a;
      f.side = s;
      F.push_back(f);
    }
  for (int q = 0; q < nh; ++q) {
    HFeat f{D == 2 ? T_C : T_S, D - 1, K_HOLE};
    f.hole = q;
    F.push_back(f);
  }
  if (D == 3)
    for (int a = 0; a < 3; ++a)
      for (int q = 0; q < 4; ++q) {
        HFeat f{T_C, 1, K_EDGE3};
        f.axis = a;
        f.fax[0] = a == 0 ? 1 : 0;
        f.fax[1] = a == 2 ? 1 : 2;
        f.fsd[0] = q & 1;
        f.fsd[1] = (q >> 1) & 1;
        F.push_back(f);
      }
  for (int c = 0; c < (1 << D); ++c) {
    HFeat f{T_SI, 0, K_CORNER};
    f.bits = c;
    F.push_back(f);
  }
  return F;
}

// does the lower-dimensional feature B lie on the boundary of feature A?
bool on_boundary_of(const HFeat &A, const HFeat &B) {
  if (B.k >= A.k) return false;
  if (A.kind == K_VOL) return true;
  if (A.kind == K_BOXSIDE) {
    if (B.kind == K_CORNER) return ((B.bits >> A.axis) & 1) == A.side;
    if (B.kind == K_EDGE3)
      return (B.fax[0] == A.axis && B.fsd[0] == A.side) || (B.fax[1] == A.axis && B.fsd[1] == A.side);
    return false;
  }
  if (A.kind == K_EDGE3 && B.kind == K_CORNER)
    return ((B.bits >> A.fax[0]) & 1) == A.fsd[0] && ((B.bits >> A.fax[1]) & 1) == A.fsd[1];
  return false;
}

// outward normal of A's boundary at a particle of B (constant unless B is a hole)
BNorm boundary_normal(int D, const HFeat &A, const HFeat &B) {
  BNorm N{};
  if (!on_boundary_of(A, B)) return N;
  N.mode = 1;
  auto sg = [](int s) { return s ? 1.0 : -1.0; };
  if (A.kind == K_VOL) {
    if (B.kind == K_BOXSIDE) {
      N.n[B.axis] = sg(B.side);
    } else if (B.kind == K_HOLE) {
      N.mode = 2;
      N.hole = B.hole;
    } else if (B.kind == K_EDGE3) {
      const double r = std::sqrt(0.5);
      N.n[B.fax[0]] = sg(B.fsd[0]) * r;
      N.n[B.fax[1]] = sg(B.fsd[1]) * r;
    } else if (B.kind == K_CORNER) {
      const double r = 1.0 / std::sqrt((double)D);
      for (int a = 0; a < D; ++a) N.n[a] = sg((B.bits >> a) & 1) * r;
    }
  } else if (A.kind == K_BOXSIDE && D == 3) {
    if (B.kind == K_EDGE3) {
      const int o = B.fax[0] == A.axis ? 1 : 0;
      N.n[B.fax[o]] = sg(B.fsd[o]);
    } else {
      const double r = std::sqrt(0.5);
      for (int a = 0; a < 3; ++a)
        if (a != A.axis) N.n[a] = sg((B.bits >> a) & 1) * r;
    }
  } else if (A.kind == K_BOXSIDE) {
    const int o = 1 - A.axis;
    N.n[o] = sg((B.bits >> o) & 1);
  } else if (A.kind == K_EDGE3) {
    N.n[A.axis] = sg((B.bits >> A.axis) & 1);
  }
  return N;
}

template <typename T>
T *dalloc(size_t count, std::vector<void *> &owned, size_t &bytes) {
  void *p = nullptr;
  size_t b = std::max<size_t>(count, 1) * sizeof(T);
  b = (b + 255) & ~size_t(255);
  if (hipMalloc(&p, b) != hipSuccess) return nullptr;
  owned.push_back(p);
  bytes += b;
  return (T *)p;
}

}  // namespace

struct sph_mesh {
  int D = 2, n = 0, nf = 0, prec = SPH_FP64, cap = 64, bw = 0;
  double p0 = 1.0;
  Geom geom{};
  Grid grid{};
  Ctl ctl{};
  std::vector<HFeat> feats;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  bool use_graph = false, debug = false;
  // device memory
  std::vector<void *> owned;
  size_t bytes = 0;
  Parts P[2]{};
  int cur = 0;
  uint32_t *cell = nullptr, *rank = nullptr, *psrc = nullptr, *pkey = nullptr;
  uint32_t *cnt = nullptr, *cstart = nullptr, *ticket = nullptr;
  unsigned long long *scan_status = nullptr;
  uint32_t *nbr = nullptr, *nnb = nullptr;
  void *ap = nullptr, *acc = nullptr;              // {ax, ay, az, 0} in the sweep precision
  double *dbg_gam = nullptr, *dbg_vt = nullptr;
  double4 *dbg_vm = nullptr;
  Feat *d_feat = nullptr;
  BNorm *d_bn = nullptr;
  int8_t *d_rel = nullptr;
  unsigned long long *d_bmask = nullptr;   // per feature: bit f set if feature f bounds it
  Group *d_grp = nullptr;
  Status *d_st = nullptr;
  uint32_t nscan_tiles = 0;
  int nblk = 0;                                 // particle blocks of one launch
  int nblk8 = 0;                                // rounded up to the 8 XCDs
  unsigned long long *pmin = nullptr, *psum = nullptr, *pcount = nullptr, *pesc = nullptr;
  // graph of two steps
  hipGraphExec_t gexec = nullptr;
  // profiling
  bool profiling = false;
  struct Ev { int kid; hipEvent_t a, b; };
  std::vector<Ev> ev_live;
  std::vector<hipEvent_t> ev_pool;
  double kms[KID_COUNT] = {};
  long long kcount[KID_COUNT] = {};

  ~sph_mesh() {
    if (stream) (void)hipStreamSynchronize(stream);
    if (gexec) (void)hipGraphExecDestroy(gexec);
    for (auto &e : ev_live) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
    for (auto e : ev_pool) (void)hipEventDestroy(e);
    for (void *p : owned) (void)hipFree(p);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }

  hipEvent_t get_event() {
    if (!ev_pool.empty()) {
      hipEvent_t e = ev_pool.back();
      ev_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }

  template <typename K, typename... A>
  hipError_t launch(int kid, K kern, unsigned grid, unsigned block, A... args) {
    if (grid == 0) return hipSuccess;
    hipEvent_t a = nullptr, b = nullptr;
    if (profiling) {
      a = get_event();
      (void)hipEventRecord(a, stream);
    }
    hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, stream, args...);
    hipError_t e = hipGetLastError();
    if (profiling) {
      b = get_event();
      (void)hipEventRecord(b, stream);
      ev_live.push_back({kid, a, b});
    }
    return e;
  }

  unsigned blocks(size_t count) const { return (unsigned)((count + BLOCK - 1) / BLOCK); }

  template <int DD>
  sph_status enqueue_hash() {
    HIPCHK(launch(KID_HASH, k_hash<DD>, blocks(n), BLOCK, geom, grid, P[cur], n, cell, rank, cnt));
    return SPH_OK;
  }

  // counting sort of the current particles into (cell, caller id) order;
  // needs cell / rank / cnt of the current buffer, leaves cnt cleared
  sph_status enqueue_sort() {
    HIPCHK(launch(KID_SCAN, k_scan, nscan_tiles, BLOCK, (const uint32_t *)cnt, cstart, grid.ncell,
                  scan_status, ticket, nscan_tiles, d_st));
    HIPCHK(launch(KID_SCATTER, k_scatter, blocks(n), BLOCK, n, (const uint32_t *)cell,
                  (const uint32_t *)rank, (const uint32_t *)cstart, (const uint32_t *)P[cur].oid,
                  psrc, pkey, scan_status, nscan_tiles, ticket));
    HIPCHK(launch(KID_RANK_GATHER, k_rank_gather, blocks(n), BLOCK, n, (const uint32_t *)psrc,
                  (const uint32_t *)pkey, (const uint32_t *)cell, (const uint32_t *)cstart, cnt,
                  P[cur], P[1 - cur]));
    cur = 1 - cur;
    return SPH_OK;
  }

  template <int DD>
  sph_status enqueue_lists_only() {
    HIPCHK(launch(KID_NBR_LISTS, k_nbr_forces<DD, double, false>, (unsigned)nblk8, BLOCK, geom,
                  grid, p0, bw, P[cur], n, (const uint32_t *)cstart, (const unsigned long long *)d_bmask,
                  (const Feat *)d_feat, (const BNorm *)d_bn, (const Group *)d_grp, 1, nbr, nnb, cap,
                  d_st, (double4 *)nullptr, (double *)nullptr, (double *)nullptr,
                  (unsigned long long *)nullptr, (unsigned long long *)nullptr,
                  (unsigned long long *)nullptr));
    return SPH_OK;
  }

  template <int DD, typename R>
  sph_status enqueue_forces() {
    using R4 = typename Vec4<R>::T;
    Parts &s = P[cur];
    HIPCHK(launch(KID_NBR_FORCES, k_nbr_forces<DD, R, true>, (unsigned)nblk8, BLOCK, geom, grid, p0,
                  bw, s, n, (const uint32_t *)cstart, (const unsigned long long *)d_bmask,
                  (const Feat *)d_feat,
                  (const BNorm *)d_bn, (const Group *)d_grp, 0, nbr, nnb, cap, d_st, (R4 *)ap,
                  dbg_gam, dbg_vt, pmin, psum, pcount));
    HIPCHK(launch(KID_REDUCE_A, k_group_reduce, (unsigned)nf, BLOCK,
                  (const unsigned long long *)pmin, (const unsigned long long *)psum, nblk8, nf,
                  ctl.dt_max, d_grp, 0));
    HIPCHK(launch(KID_SWEEP_B, k_sweep_b<DD, R>, (unsigned)nblk8, BLOCK, geom, s, n,
                  (const uint32_t *)nbr, (const uint32_t *)nnb, (const Feat *)d_feat,
                  (const Group *)d_grp, (const R4 *)ap, (R4 *)acc, dbg_vm, pmin));
    HIPCHK(launch(KID_REDUCE_B, k_group_reduce, (unsigned)nf, BLOCK,
                  (const unsigned long long *)pmin, (const unsigned long long *)nullptr, nblk8, nf,
                  ctl.dt_max, d_grp, 1));
    HIPCHK(launch(KID_INTEGRATE_HASH, k_integrate_hash<DD, R>, blocks(n), BLOCK, geom, grid, s, n,
                  (const Feat *)d_feat, (const Group *)d_grp, (const R4 *)acc, d_st, pesc, cell,
                  rank, cnt));
    HIPCHK(launch(KID_CONTROL, k_control, 1u, BLOCK, ctl, d_grp, nf, d_st,
                  (const unsigned long long *)pcount, nblk8, (const unsigned long long *)pesc,
                  nblk));
    return SPH_OK;
  }

  sph_status enqueue_step() {
    if (sph_status st = enqueue_sort()) return st;
    if (D == 2) return prec == SPH_FP64 ? enqueue_forces<2, double>() : enqueue_forces<2, float>();
    return prec == SPH_FP64 ? enqueue_forces<3, double>() : enqueue_forces<3, float>();
  }

  sph_status hash_now() { return D == 2 ? enqueue_hash<2>() : enqueue_hash<3>(); }

  sph_status build_graph() {
    if (gexec) return SPH_OK;
    const int saved = cur;
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
    sph_status st = enqueue_step();
    if (!st) st = enqueue_step();
    hipError_t e = hipStreamEndCapture(stream, &graph);
    cur = saved;
    if (st) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    if (e != hipSuccess) return fail(SPH_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      gexec = nullptr;
      return fail(SPH_ERR_DEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
    }
    return SPH_OK;
  }

  sph_status check_status() {
    Status s{};
    HIPCHK(hipMemcpy(&s, d_st, sizeof s, hipMemcpyDeviceToHost));
    if (s.nan_flag) return fail(SPH_ERR_STATE, "non-finite position of particle %u", s.nan_oid);
    if (s.scan_fail) return fail(SPH_ERR_DEVICE, "cell-count scan lost a tile");
    if (s.overflow)
      return fail(SPH_ERR_STATE, "neighbour list overflow: %u neighbours > capacity %d "
                                 "(raise max_neighbors)", s.overflow_max, cap);
    return SPH_OK;
  }
};

// ---------------------------------------------------------------------------
// creation
// ---------------------------------------------------------------------------
static sph_status validate(const sph_geometry *g, const sph_sizing *s, const sph_params *p) {
  if (!g || !s || !p) return fail(SPH_ERR_INVALID_ARG, "null geometry, sizing or params");
  if (g->dim != 2 && g->dim != 3) return fail(SPH_ERR_INVALID_ARG, "dim must be 2 or 3");
  for (int a = 0; a < g->dim; ++a)
    if (!(g->lo[a] < g->hi[a]) || !std::isfinite(g->lo[a]) || !std::isfinite(g->hi[a]))
      return fail(SPH_ERR_INVALID_ARG, "empty or non-finite box on axis %d", a);
  if (g->n_holes < 0 || g->n_holes > MAXH)
    return fail(SPH_ERR_INVALID_ARG, "n_holes must be in [0, %d]", MAXH);
  if (g->n_holes > 0 && !g->holes) return fail(SPH_ERR_INVALID_ARG, "holes is NULL");
  for (int q = 0; q < g->n_holes; ++q) {
    const double *H = g->holes + 15 * q;
    if (!(H[3] > 0) || H[4] != H[3] || H[5] != H[3])
      return fail(SPH_ERR_UNSUPPORTED, "hole %d: only discs / balls (equal semi-axes)", q);
    for (int a = 0; a < g->dim; ++a)
      if (!(H[a] - H[3] > g->lo[a] && H[a] + H[3] < g->hi[a]))
        return fail(SPH_ERR_INVALID_ARG, "hole %d must lie strictly inside the box", q);
  }
  if (s->kind < 0 || s->kind > 2) return fail(SPH_ERR_INVALID_ARG, "unknown sizing kind");
  if (!(s->h0 > 0) || !(s->grad >= 0) || !std::isfinite(s->h0) || !std::isfinite(s->grad))
    return fail(SPH_ERR_INVALID_ARG, "sizing needs h0 > 0 and grad >= 0");
  if (s->kind == 2 && g->n_holes == 0 && !std::isfinite(s->dcap))
    return fail(SPH_ERR_INVALID_ARG, "graded sizing without holes needs a finite dcap");
  if (!(s->dcap >= 0)) return fail(SPH_ERR_INVALID_ARG, "dcap must be >= 0");
  if (p->window_samples < 1 || p->window_samples > MAXRING || p->sample_every < 1 ||
      p->reset_period < 1 || p->ramp_halving < 1 || p->ramp_steps < 1 || p->phase2_steps < 0 ||
      p->max_phase1_steps < 1)
    return fail(SPH_ERR_INVALID_ARG, "bad control parameters");
  if (!(p->dt_max > 0) || !(p->tol >= 0) || !std::isfinite(p->p0) || !(p->p0 > 0))
    return fail(SPH_ERR_INVALID_ARG, "need dt_max > 0, tol >= 0, p0 > 0");
  if (p->boundary_weighting < 0 || p->boundary_weighting > 2)
    return fail(SPH_ERR_INVALID_ARG, "boundary_weighting must be 0, 1 or 2");
  if (p->precision != SPH_FP64 && p->precision != SPH_FP32_MIXED)
    return fail(SPH_ERR_INVALID_ARG, "precision must be SPH_FP64 or SPH_FP32_MIXED");
  if (p->max_neighbors < 0 || p->max_neighbors > 4096)
    return fail(SPH_ERR_INVALID_ARG, "max_neighbors must be in [0, 4096]");
  return SPH_OK;
}

// bounds of h_t over the box (points outside every hole), and its Lipschitz constant
static void sizing_bounds(const sph_geometry *g, const sph_sizing *s, double &hmin, double &hmax,
                          double &lip) {
  const int D = g->dim;
  auto corner = [&](int c, int a) { return ((c >> a) & 1) ? g->hi[a] : g->lo[a]; };
  hmin = s->h0;
  if (s->kind == 0) {
    hmax = s->h0;
    lip = 0.0;
    return;
  }
  if (s->kind == 1) {
    double far = 0.0;
    for (int c = 0; c < (1 << D); ++c) {
      double d2 = 0.0;
      for (int a = 0; a < D; ++a) d2 += (corner(c, a) - s->point[a]) * (corner(c, a) - s->point[a]);
      far = std::max(far, std::sqrt(d2));
    }
    hmax = s->h0 + s->grad * far;
    lip = s->grad;
    return;
  }
  // graded to holes: d(x) <= distance to hole q <= farthest box corner - r_q
  double dmax = s->dcap;
  for (int q = 0; q < g->n_holes; ++q) {
    const double *H = g->holes + 15 * q;
    double far = 0.0;
    for (int c = 0; c < (1 << D); ++c) {
      double d2 = 0.0;
      for (int a = 0; a < D; ++a) d2 += (corner(c, a) - H[a]) * (corner(c, a) - H[a]);
      far = std::max(far, std::sqrt(d2));
    }
    dmax = std::min(dmax, far - H[3]);
  }
  hmax = s->h0 * (1.0 + s->grad * dmax);
  lip = s->h0 * s->grad;
}

extern "C" sph_status sph_mesh_create(const sph_geometry *g, const sph_sizing *s,
                                      const sph_params *p, int64_t n, const double *xyz,
                                      const int32_t *feature, sph_mesh **out) {
  if (!out) return fail(SPH_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (sph_status st = validate(g, s, p)) return st;
  if (n < 0 || n > 0x7fffffff || (n > 0 && (!xyz || !feature)))
    return fail(SPH_ERR_INVALID_ARG, "bad particle count or NULL particle arrays");
  const int D = g->dim;
  auto feats = make_features(D, g->n_holes);
  const int nf = (int)feats.size();
  if (nf > MAXF) return fail(SPH_ERR_UNSUPPORTED, "too many features (%d > %d)", nf, MAXF);
  for (int64_t i = 0; i < n; ++i)
    if (feature[i] < 0 || feature[i] >= nf)
      return fail(SPH_ERR_INVALID_ARG, "particle %lld: feature %d out of range [0, %d)",
                  (long long)i, feature[i], nf);

  auto *M = new sph_mesh();
  M->D = D;
  M->n = (int)n;
  M->nf = nf;
  M->feats = feats;
  M->prec = p->precision;
  M->cap = p->max_neighbors ? p->max_neighbors : (D == 2 ? 64 : 160);
  M->bw = p->boundary_weighting;
  M->p0 = p->p0;
  M->use_graph = p->use_graph != 0;
  M->debug = p->debug_fields != 0;
  // geometry + sizing record
  Geom &G = M->geom;
  G.dim = D;
  G.nf = nf;
  G.nh = g->n_holes;
  G.hkind = s->kind;
  for (int a = 0; a < 3; ++a) {
    G.lo[a] = g->lo[a];
    G.hi[a] = g->hi[a];
    G.hpt[a] = s->point[a];
  }
  for (int q = 0; q < g->n_holes; ++q) {
    for (int a = 0; a < 3; ++a) G.hc[q][a] = g->holes[15 * q + a];
    G.hr[q] = g->holes[15 * q + 3];
  }
  G.h0 = s->h0;
  G.grad = s->grad;
  G.dcap = s->dcap;
  // control
  Ctl &C = M->ctl;
  C.tol = p->tol;
  C.eps_damp = p->eps_damp;
  C.dt_max = p->dt_max;
  C.reset_period = p->reset_period;
  C.sample_every = p->sample_every;
  C.window_samples = p->window_samples;
  C.ramp_steps = p->ramp_steps;
  C.ramp_halving = p->ramp_halving;
  C.phase2_steps = p->phase2_steps;
  C.max_phase1_steps = p->max_phase1_steps;
  // cell grid: side 2 h_min cell_factor; search radius from the Lipschitz bound
  double hmin, hmax, lip;
  sizing_bounds(g, s, hmin, hmax, lip);
  Grid &Gr = M->grid;
  const double cf = p->cell_factor > 0 ? p->cell_factor : 1.0;
  double side = 2.0 * hmin * cf;
  for (;;) {
    double cells = 1.0;
    for (int a = 0; a < D; ++a) cells *= std::max(1.0, std::floor((g->hi[a] - g->lo[a]) / side));
    if (cells <= 16.0 * 1024 * 1024) break;
    side *= 1.25;
  }
  Gr.ncell = 1;
  for (int a = 0; a < 3; ++a) {
    Gr.lo[a] = g->lo[a];
    if (a < D) {
      Gr.nc[a] = (int)std::max(1.0, std::floor((g->hi[a] - g->lo[a]) / side));
      Gr.inv_c[a] = Gr.nc[a] / (g->hi[a] - g->lo[a]);
      Gr.c[a] = (g->hi[a] - g->lo[a]) / Gr.nc[a];
    } else {
      Gr.nc[a] = 1;
      Gr.inv_c[a] = 0.0;
      Gr.c[a] = 0.0;
    }
    Gr.ncell *= (uint32_t)Gr.nc[a];
  }
  Gr.rmax = 2.0 * hmax * (1.0 + 1e-9);
  Gr.rfac = 2.0 * lip < 0.9 ? 2.0 * (1.0 + 1e-9) / (1.0 - 2.0 * lip) : 1e300;
  M->nscan_tiles = (Gr.ncell + SCAN_TILE - 1) / SCAN_TILE;

  // stream
  if (p->stream) {
    M->stream = (hipStream_t)p->stream;
  } else {
    if (hipStreamCreateWithFlags(&M->stream, hipStreamNonBlocking) != hipSuccess) {
      delete M;
      return fail(SPH_ERR_DEVICE, "hipStreamCreate failed");
    }
    M->own_stream = true;
  }

  // device memory
  auto &ow = M->owned;
  size_t &by = M->bytes;
  const size_t N = (size_t)n;
  bool ok = true;
  // records are padded past n so that batched candidate loads need no clamp
  const size_t NPAD = N + 8;
  for (int b = 0; b < 2; ++b) {
    M->P[b].xh = dalloc<double4>(NPAD, ow, by);
    M->P[b].v = dalloc<double4>(NPAD, ow, by);
    M->P[b].f = dalloc<uint8_t>(NPAD, ow, by);
    M->P[b].oid = dalloc<uint32_t>(N, ow, by);
    ok = ok && M->P[b].xh && M->P[b].v && M->P[b].f && M->P[b].oid;
  }
  M->cell = dalloc<uint32_t>(N, ow, by);
  M->rank = dalloc<uint32_t>(N, ow, by);
  M->psrc = dalloc<uint32_t>(N, ow, by);
  M->pkey = dalloc<uint32_t>(N, ow, by);
  M->cnt = dalloc<uint32_t>(Gr.ncell, ow, by);
  M->cstart = dalloc<uint32_t>((size_t)Gr.ncell + 1, ow, by);
  M->scan_status = dalloc<unsigned long long>(M->nscan_tiles, ow, by);
  M->ticket = dalloc<uint32_t>(1, ow, by);
  M->nbr = dalloc<uint32_t>(N * (size_t)M->cap, ow, by);
  M->nnb = dalloc<uint32_t>(N, ow, by);
  const size_t r4 = M->prec == SPH_FP64 ? sizeof(double4) : sizeof(float4);
  M->ap = dalloc<char>(N * r4, ow, by);
  M->acc = dalloc<char>(N * r4, ow, by);
  ok = ok && M->ap && M->acc;
  if (M->debug) {
    M->dbg_gam = dalloc<double>(N, ow, by);
    M->dbg_vt = dalloc<double>(N, ow, by);
    M->dbg_vm = dalloc<double4>(N, ow, by);
    ok = ok && M->dbg_gam && M->dbg_vt && M->dbg_vm;
  }
  M->d_feat = dalloc<Feat>(nf, ow, by);
  M->d_bn = dalloc<BNorm>((size_t)nf * nf, ow, by);
  M->d_rel = dalloc<int8_t>((size_t)nf * nf, ow, by);
  M->d_bmask = dalloc<unsigned long long>(nf, ow, by);
  M->d_grp = dalloc<Group>(nf, ow, by);
  M->d_st = dalloc<Status>(1, ow, by);
  M->nblk = (int)((N + BLOCK - 1) / BLOCK);
  M->nblk8 = (M->nblk + 7) / 8 * 8;
  M->pmin = dalloc<unsigned long long>((size_t)std::max(M->nblk8, 1) * nf, ow, by);
  M->psum = dalloc<unsigned long long>((size_t)std::max(M->nblk8, 1) * nf, ow, by);
  M->pcount = dalloc<unsigned long long>(std::max(M->nblk8, 1), ow, by);
  M->pesc = dalloc<unsigned long long>(std::max(M->nblk, 1), ow, by);
  ok = ok && M->pmin && M->psum && M->pcount && M->pesc && M->cell && M->rank && M->psrc && M->pkey && M->cnt && M->cstart &&
       M->scan_status && M->ticket && M->nbr && M->nnb && M->d_feat && M->d_bn && M->d_rel && M->d_bmask && M->d_grp && M->d_st;
  if (!ok) {
    delete M;
    return fail(SPH_ERR_OUT_OF_MEMORY, "device allocation of %zu bytes failed", by);
  }

  // host-side tables
  std::vector<Feat> hf(nf);
  std::vector<BNorm> hb((size_t)nf * nf);
  std::vector<int8_t> hr((size_t)nf * nf, 0);
  std::vector<unsigned long long> hm(nf, 0ull);
  for (int i = 0; i < nf; ++i) {
    const HFeat &F = feats[i];
    Feat d{};
    d.type = (int8_t)F.type;
    d.k = (int8_t)F.k;
    d.kind = (int8_t)F.kind;
    d.axis = (int8_t)F.axis;
    d.side = (int8_t)F.side;
    d.fax0 = (int8_t)F.fax[0];
    d.fsd0 = (int8_t)F.fsd[0];
    d.fax1 = (int8_t)F.fax[1];
    d.fsd1 = (int8_t)F.fsd[1];
    d.hole = (int8_t)F.hole;
    d.bits = (int8_t)F.bits;
    hf[i] = d;
    for (int j = 0; j < nf; ++j) {
      hb[(size_t)i * nf + j] = boundary_normal(D, F, feats[j]);
      hr[(size_t)i * nf + j] = i == j ? 1 : (on_boundary_of(F, feats[j]) ? 2 : 0);
      if (i != j && on_boundary_of(F, feats[j])) hm[i] |= 1ull << j;
    }
  }
  std::vector<int64_t> counts(nf, 0);
  for (int64_t i = 0; i < n; ++i) counts[feature[i]]++;
  std::vector<Group> hg(nf);
  for (int q = 0; q < nf; ++q) {
    Group &Q = hg[q];
    std::memset(&Q, 0, sizeof Q);
    Q.tracked = feats[q].type != T_SI && counts[q] > 0;
    Q.active = Q.tracked;
    Q.phase = PH_ONE;
    Q.count = (int32_t)counts[q];
    Q.eps = p->eps_damp;
    Q.esys = HUGE_VAL;
    double db = p->dt_max;
    std::memcpy(&Q.dt1_bits, &db, 8);
    std::memcpy(&Q.dt_bits, &db, 8);
    // fixed-point scale of the V~ sum: V~_i <= h^k / alpha_k, keep the
    // group total below 2^62
    const int k = feats[q].k;
    const double alpha = k == 1 ? 0.625 : (k == 2 ? 7.0 / (4.0 * M_PI) : 21.0 / (16.0 * M_PI));
    double bound = (double)std::max<int64_t>(counts[q], 1) * std::pow(hmax, k) / alpha;
    int e = 62 - (int)std::ceil(std::log2(bound * 2.0));
    Q.vscale = std::ldexp(1.0, std::min(e, 1000));
  }
  // particle records: caller order, caller ids
  std::vector<double4> xh(N);
  std::vector<uint32_t> oid(N);
  std::vector<uint8_t> f8(N);
  for (size_t i = 0; i < N; ++i) {
    xh[i] = make_double4(xyz[3 * i], xyz[3 * i + 1], D == 3 ? xyz[3 * i + 2] : 0.0, 0.0);
    oid[i] = (uint32_t)i;
    f8[i] = (uint8_t)feature[i];
  }
  hipError_t e = hipSuccess;
  if (N) e = hipMemcpy(M->P[0].xh, xh.data(), N * sizeof(double4), hipMemcpyHostToDevice);
  if (e == hipSuccess && N) e = hipMemset(M->P[0].v, 0, N * sizeof(double4));
  if (e == hipSuccess && N) e = hipMemcpy(M->P[0].oid, oid.data(), N * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess && N) e = hipMemcpy(M->P[0].f, f8.data(), N, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(M->d_feat, hf.data(), sizeof(Feat) * nf, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(M->d_bn, hb.data(), sizeof(BNorm) * nf * nf, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(M->d_rel, hr.data(), (size_t)nf * nf, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(M->d_bmask, hm.data(), 8 * nf, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(M->d_grp, hg.data(), sizeof(Group) * nf, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(M->d_st, 0, sizeof(Status));
  if (e == hipSuccess) e = hipMemset(M->cnt, 0, sizeof(uint32_t) * Gr.ncell);
  if (e == hipSuccess)
    e = hipMemset(M->scan_status, 0, sizeof(unsigned long long) * std::max(M->nscan_tiles, 1u));
  if (e == hipSuccess) e = hipMemset(M->ticket, 0, sizeof(uint32_t));
  if (e == hipSuccess) e = hipMemset(M->nnb, 0, sizeof(uint32_t) * std::max<size_t>(N, 1));
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    delete M;
    return fail(SPH_ERR_DEVICE, "initial upload failed: %s", hipGetErrorString(e));
  }
  if (N) {
    if (sph_status st = M->hash_now()) {
      delete M;
      return st;
    }
    if ((e = hipStreamSynchronize(M->stream)) != hipSuccess) {
      delete M;
      return fail(SPH_ERR_DEVICE, "initial hash failed: %s", hipGetErrorString(e));
    }
  }
  *out = M;
  return SPH_OK;
}

extern "C" void sph_mesh_destroy(sph_mesh *m) { delete m; }

extern "C" const char *sph_mesh_last_error(void) { return g_err.c_str(); }

extern "C" sph_status sph_mesh_step(sph_mesh *m, int32_t n_steps) {
  if (!m || n_steps < 0) return fail(SPH_ERR_INVALID_ARG, "bad handle or step count");
  if (m->n == 0) return SPH_OK;
  int left = n_steps;
  if (m->use_graph && !m->profiling) {
    if (left > 0 && m->cur != 0) {   // graphs are captured at parity 0
      if (sph_status st = m->enqueue_step()) return st;
      --left;
    }
    if (left >= 2) {
      if (sph_status st = m->build_graph()) return st;
      for (; left >= 2; left -= 2) HIPCHK(hipGraphLaunch(m->gexec, m->stream));
    }
  }
  for (; left > 0; --left)
    if (sph_status st = m->enqueue_step()) return st;
  return SPH_OK;
}

extern "C" sph_status sph_mesh_sync(sph_mesh *m) {
  if (!m) return fail(SPH_ERR_INVALID_ARG, "null handle");
  HIPCHK(hipStreamSynchronize(m->stream));
  return SPH_OK;
}

// copy a device column (slot order) to a host vector
template <typename T>
static hipError_t pull(std::vector<T> &h, const void *d, size_t count) {
  h.resize(count);
  if (!count) return hipSuccess;
  return hipMemcpy(h.data(), d, count * sizeof(T), hipMemcpyDeviceToHost);
}

extern "C" sph_status sph_mesh_positions(sph_mesh *m, double *xyz, int32_t *feature,
                                         int64_t capacity, int64_t *n_out) {
  if (!m) return fail(SPH_ERR_INVALID_ARG, "null handle");
  if (n_out) *n_out = m->n;
  if (!xyz && !feature) return SPH_OK;
  if (capacity < m->n) return fail(SPH_ERR_INVALID_ARG, "capacity %lld < %d particles",
                                   (long long)capacity, m->n);
  HIPCHK(hipStreamSynchronize(m->stream));
  if (sph_status st = m->check_status()) return st;
  const Parts &s = m->P[m->cur];
  std::vector<uint32_t> oid;
  HIPCHK(pull(oid, s.oid, m->n));
  if (xyz) {
    std::vector<double4> xh;
    HIPCHK(pull(xh, s.xh, m->n));
    for (int i = 0; i < m->n; ++i) {
      double *o = xyz + 3 * (size_t)oid[i];
      o[0] = xh[i].x;
      o[1] = xh[i].y;
      o[2] = m->D == 3 ? xh[i].z : 0.0;
    }
  }
  if (feature) {
    std::vector<uint8_t> f;
    HIPCHK(pull(f, s.f, m->n));
    for (int i = 0; i < m->n; ++i) feature[oid[i]] = f[i];
  }
  return SPH_OK;
}

extern "C" sph_status sph_mesh_velocities(sph_mesh *m, double *vel) {
  if (!m || !vel) return fail(SPH_ERR_INVALID_ARG, "null argument");
  HIPCHK(hipStreamSynchronize(m->stream));
  const Parts &s = m->P[m->cur];
  std::vector<uint32_t> oid;
  HIPCHK(pull(oid, s.oid, m->n));
  std::vector<double4> v;
  HIPCHK(pull(v, s.v, m->n));
  for (int i = 0; i < m->n; ++i) {
    double *o = vel + 3 * (size_t)oid[i];
    o[0] = v[i].x;
    o[1] = v[i].y;
    o[2] = m->D == 3 ? v[i].z : 0.0;
  }
  return SPH_OK;
}

extern "C" sph_status sph_mesh_set_state(sph_mesh *m, const double *xyz, const double *vel) {
  if (!m) return fail(SPH_ERR_INVALID_ARG, "null handle");
  HIPCHK(hipStreamSynchronize(m->stream));
  if (m->n == 0) return SPH_OK;
  const Parts &s = m->P[m->cur];
  std::vector<uint32_t> oid;
  HIPCHK(pull(oid, s.oid, m->n));
  if (xyz) {
    std::vector<double4> xh(m->n);
    for (int i = 0; i < m->n; ++i) {
      const double *p = xyz + 3 * (size_t)oid[i];
      xh[i] = make_double4(p[0], p[1], m->D == 3 ? p[2] : 0.0, 0.0);
    }
    HIPCHK(hipMemcpy(s.xh, xh.data(), xh.size() * sizeof(double4), hipMemcpyHostToDevice));
    // new positions: new h, cells and ranks
    HIPCHK(hipMemset(m->cnt, 0, sizeof(uint32_t) * m->grid.ncell));
    if (sph_status st = m->hash_now()) return st;
    HIPCHK(hipStreamSynchronize(m->stream));
  }
  if (vel) {
    std::vector<double4> v(m->n);
    for (int i = 0; i < m->n; ++i) {
      const double *p = vel + 3 * (size_t)oid[i];
      v[i] = make_double4(p[0], p[1], m->D == 3 ? p[2] : 0.0, 0.0);
    }
    HIPCHK(hipMemcpy(s.v, v.data(), v.size() * sizeof(double4), hipMemcpyHostToDevice));
  }
  return SPH_OK;
}

extern "C" sph_status sph_mesh_neighbors(sph_mesh *m, int64_t *offsets, int32_t *ids, int8_t *rel,
                                         int64_t cap, int64_t *n_pairs) {
  if (!m || !offsets) return fail(SPH_ERR_INVALID_ARG, "null argument");
  HIPCHK(hipStreamSynchronize(m->stream));
  const int n = m->n;
  if (n == 0) {
    offsets[0] = 0;
    if (n_pairs) *n_pairs = 0;
    return SPH_OK;
  }
  // sort into cell order, build the lists, then re-hash so that the next
  // step starts from consistent cell counts
  sph_status st = m->enqueue_sort();
  if (!st) st = m->D == 2 ? m->enqueue_lists_only<2>() : m->enqueue_lists_only<3>();
  if (!st) st = m->hash_now();
  if (st) return st;
  HIPCHK(hipStreamSynchronize(m->stream));
  if ((st = m->check_status())) return st;
  const Parts &s = m->P[m->cur];
  std::vector<uint32_t> oid, nnb, nbr;
  HIPCHK(pull(oid, s.oid, n));
  HIPCHK(pull(nnb, m->nnb, n));
  HIPCHK(pull(nbr, m->nbr, (size_t)n * m->cap));
  std::vector<int64_t> cnt(n + 1, 0);
  for (int i = 0; i < n; ++i) cnt[oid[i] + 1] = nnb[i];
  for (int i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
  std::memcpy(offsets, cnt.data(), sizeof(int64_t) * (n + 1));
  if (n_pairs) *n_pairs = cnt[n];
  if (!ids && !rel) return SPH_OK;
  if (cap < cnt[n]) return fail(SPH_ERR_INVALID_ARG, "capacity %lld < %lld pairs", (long long)cap,
                                (long long)cnt[n]);
  std::vector<std::pair<uint32_t, int8_t>> tmp;
  for (int i = 0; i < n; ++i) {
    tmp.clear();
    for (uint32_t e = 0; e < nnb[i]; ++e) {
      uint32_t u = nbr[(size_t)e * n + i];
      tmp.push_back({oid[u & 0x7fffffffu], (int8_t)((u >> 31) ? 2 : 1)});
    }
    std::sort(tmp.begin(), tmp.end());
    int64_t o = cnt[oid[i]];
    for (size_t t = 0; t < tmp.size(); ++t) {
      if (ids) ids[o + t] = (int32_t)tmp[t].first;
      if (rel) rel[o + t] = tmp[t].second;
    }
  }
  return SPH_OK;
}

extern "C" sph_status sph_mesh_field(sph_mesh *m, int32_t which, double *out) {
  if (!m || !out) return fail(SPH_ERR_INVALID_ARG, "null argument");
  if (which < 0 || which > 5) return fail(SPH_ERR_INVALID_ARG, "unknown field %d", which);
  if (which >= 3 && !m->debug) return fail(SPH_ERR_INVALID_ARG, "field %d needs debug_fields", which);
  HIPCHK(hipStreamSynchronize(m->stream));
  const int n = m->n;
  const Parts &s = m->P[m->cur];
  std::vector<uint32_t> oid;
  HIPCHK(pull(oid, s.oid, n));
  std::vector<double> col;
  auto scatter1 = [&]() {
    for (int i = 0; i < n; ++i) out[oid[i]] = col[i];
  };
  auto scatter4 = [&](const std::vector<double4> &v) {
    for (int i = 0; i < n; ++i) {
      double *o = out + 3 * (size_t)oid[i];
      o[0] = v[i].x;
      o[1] = v[i].y;
      o[2] = m->D == 3 ? v[i].z : 0.0;
    }
  };
  std::vector<double4> v4;
  switch (which) {
    case 0: {
      HIPCHK(pull(v4, s.xh, n));
      col.resize(n);
      for (int i = 0; i < n; ++i) col[i] = v4[i].w;
      scatter1();
      break;
    }
    case 3: HIPCHK(pull(col, m->dbg_vt, n)); scatter1(); break;
    case 4: HIPCHK(pull(col, m->dbg_gam, n)); scatter1(); break;
    case 5: HIPCHK(pull(v4, m->dbg_vm, n)); scatter4(v4); break;
    default: {
      const void *src = which == 1 ? m->ap : m->acc;
      if (m->prec == SPH_FP64) {
        HIPCHK(pull(v4, src, n));
      } else {
        std::vector<float4> f4;
        HIPCHK(pull(f4, src, n));
        v4.resize(n);
        for (int i = 0; i < n; ++i) v4[i] = make_double4(f4[i].x, f4[i].y, f4[i].z, f4[i].w);
      }
      scatter4(v4);
    }
  }
  return SPH_OK;
}

extern "C" sph_status sph_mesh_group_state(sph_mesh *m, int32_t f, double *out) {
  if (!m || !out || f < 0 || f >= m->nf) return fail(SPH_ERR_INVALID_ARG, "bad argument");
  HIPCHK(hipStreamSynchronize(m->stream));
  Group G;
  HIPCHK(hipMemcpy(&G, m->d_grp + f, sizeof G, hipMemcpyDeviceToHost));
  out[0] = G.phase; out[1] = G.n_ph; out[2] = G.esys; out[3] = G.dt1; out[4] = G.dt;
  out[5] = G.vbar; out[6] = G.reset_next; out[7] = G.a_last; out[8] = G.a_prev; out[9] = G.nwin;
  return SPH_OK;
}

extern "C" sph_status sph_mesh_error(sph_mesh *m, double *e_sys, int32_t *phase, int32_t *converged,
                                     int64_t *step) {
  if (!m) return fail(SPH_ERR_INVALID_ARG, "null handle");
  HIPCHK(hipStreamSynchronize(m->stream));
  if (sph_status st = m->check_status()) return st;
  std::vector<Group> G(m->nf);
  HIPCHK(hipMemcpy(G.data(), m->d_grp, sizeof(Group) * m->nf, hipMemcpyDeviceToHost));
  Status S;
  HIPCHK(hipMemcpy(&S, m->d_st, sizeof S, hipMemcpyDeviceToHost));
  double e = 0.0;
  int ph = PH_FROZEN, conv = 1;
  for (const Group &q : G) {
    if (!q.tracked) continue;
    if (q.esys > e || std::isnan(q.esys)) e = q.esys;
    ph = std::min(ph, (int)q.phase);
    if (q.phase != PH_FROZEN) conv = 0;
  }
  if (e_sys) *e_sys = e;
  if (phase) *phase = ph;
  if (converged) *converged = conv;
  if (step) *step = (int64_t)S.steps;
  return SPH_OK;
}

extern "C" sph_status sph_mesh_counters(sph_mesh *m, double *out) {
  if (!m || !out) return fail(SPH_ERR_INVALID_ARG, "null argument");
  HIPCHK(hipStreamSynchronize(m->stream));
  Status S;
  HIPCHK(hipMemcpy(&S, m->d_st, sizeof S, hipMemcpyDeviceToHost));
  out[0] = (double)S.steps;
  out[1] = (double)S.escaped;
  out[2] = (double)S.inter_total;
  out[3] = (double)S.inter_last;
  return SPH_OK;
}

extern "C" sph_status sph_mesh_control_replay(const sph_params *p, int32_t n, const double *vbar,
                                              const double *dt, int32_t *phase, int32_t *reset,
                                              double *e_sys) {
  if (!p || n < 0 || n > 1000000 || (n && (!vbar || !dt || !phase || !reset || !e_sys)))
    return fail(SPH_ERR_INVALID_ARG, "bad argument");
  if (p->window_samples < 1 || p->window_samples > MAXRING || p->sample_every < 1 ||
      p->reset_period < 1 || p->ramp_halving < 1 || p->ramp_steps < 1)
    return fail(SPH_ERR_INVALID_ARG, "bad control parameters");
  Ctl C{};
  C.tol = p->tol;
  C.eps_damp = p->eps_damp;
  C.dt_max = p->dt_max;
  C.reset_period = p->reset_period;
  C.sample_every = p->sample_every;
  C.window_samples = p->window_samples;
  C.ramp_steps = p->ramp_steps;
  C.ramp_halving = p->ramp_halving;
  C.phase2_steps = p->phase2_steps;
  C.max_phase1_steps = p->max_phase1_steps;
  Group G0;
  std::memset(&G0, 0, sizeof G0);
  G0.phase = PH_ONE;
  G0.esys = HUGE_VAL;
  G0.tracked = 1;
  void *buf = nullptr;
  const size_t nn = std::max(n, 1);
  const size_t bytes = sizeof(Group) + nn * (8 + 8 + 4 + 4 + 8);
  HIPCHK(hipMalloc(&buf, bytes));
  char *b = (char *)buf;
  Group *dg = (Group *)b;
  double *dv = (double *)(b + sizeof(Group));
  double *dd = dv + nn;
  double *de = dd + nn;
  int32_t *dp = (int32_t *)(de + nn);
  int32_t *dr = dp + nn;
  hipError_t e = hipMemcpy(dg, &G0, sizeof G0, hipMemcpyHostToDevice);
  if (e == hipSuccess && n) e = hipMemcpy(dv, vbar, n * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess && n) e = hipMemcpy(dd, dt, n * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_control_replay, dim3(1), dim3(64), 0, 0, C, n, (const double *)dv,
                       (const double *)dd, dp, dr, de, dg);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess && n) e = hipMemcpy(phase, dp, n * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess && n) e = hipMemcpy(reset, dr, n * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess && n) e = hipMemcpy(e_sys, de, n * 8, hipMemcpyDeviceToHost);
  (void)hipFree(buf);
  if (e != hipSuccess) return fail(SPH_ERR_DEVICE, "control replay: %s", hipGetErrorString(e));
  return SPH_OK;
}

extern "C" sph_status sph_mesh_profile(sph_mesh *m, int32_t enable) {
  if (!m) return fail(SPH_ERR_INVALID_ARG, "null handle");
  HIPCHK(hipStreamSynchronize(m->stream));
  for (auto &e : m->ev_live) {
    m->ev_pool.push_back(e.a);
    m->ev_pool.push_back(e.b);
  }
  m->ev_live.clear();
  for (int k = 0; k < KID_COUNT; ++k) {
    m->kms[k] = 0.0;
    m->kcount[k] = 0;
  }
  m->profiling = enable != 0;
  return SPH_OK;
}

extern "C" sph_status sph_mesh_kernel_stats(sph_mesh *m, int32_t kid, double *ms, int64_t *launches) {
  if (!m || kid < 0 || kid >= KID_COUNT) return fail(SPH_ERR_INVALID_ARG, "bad argument");
  HIPCHK(hipStreamSynchronize(m->stream));
  for (auto &e : m->ev_live) {
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, e.a, e.b));
    m->kms[e.kid] += t;
    m->kcount[e.kid] += 1;
    m->ev_pool.push_back(e.a);
    m->ev_pool.push_back(e.b);
  }
  m->ev_live.clear();
  if (ms) *ms = m->kms[kid];
  if (launches) *launches = m->kcount[kid];
  return SPH_OK;
}

extern "C" int32_t sph_mesh_kernel_count(void) { return KID_COUNT; }

extern "C" const char *sph_mesh_kernel_name(int32_t kid) {
  return kid >= 0 && kid < KID_COUNT ? kKernelNames[kid] : "";
}

extern "C" int64_t sph_mesh_device_bytes(sph_mesh *m) { return m ? (int64_t)m->bytes : 0; }
