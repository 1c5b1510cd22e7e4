// sph_mesh.hip -- host runtime and C ABI of libsphmesh.so (include/sph_mesh.h).
//
// A batch holds any number of relaxation jobs (up to 64) in one set of
// device arrays: particle columns double buffered for the per-step counting
// sort, one cell table in which every job owns a contiguous range of cells,
// one ELL neighbour list, and per-job tables of features, feature groups and
// counters.  A step is one launch sequence over all resident particles,
// whatever job they belong to, so small jobs share the chip instead of each
// filling a fraction of it.  sph_batch_step only enqueues kernels
// (optionally as a replayed HIP graph of two steps, so the double-buffer
// parity is the same at every replay); control decisions are taken on the
// device, and the host reads state back only when asked.  The single-job
// handle sph_mesh is a batch holding one job.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
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
  KID_SCAN = 0, KID_SCATTER, KID_RANK_GATHER, KID_NBR_FORCES, KID_REDUCE_A, KID_MIDPOINT,
  KID_SWEEP_B, KID_REDUCE_B, KID_INTEGRATE_HASH, KID_CONTROL, KID_HASH, KID_NBR_LISTS, KID_SKIN,
  KID_COUNT
};
const char *kKernelNames[KID_COUNT] = {
    "scan", "scatter", "rank_gather", "nbr_forces", "reduce_a", "midpoint", "sweep_b",
    "reduce_b", "integrate_hash", "control", "hash", "nbr_lists", "verlet_build"};

// ---------------------------------------------------------------------------
// features of a box-minus-holes geometry (numbering of sph_mesh.h)
// ---------------------------------------------------------------------------
struct HFeat {
  int type, k, kind, axis = 0, side = 0, fax[2] = {0, 0}, fsd[2] = {0, 0}, hole = 0, bits = 0;
  int ell = 0;   // HOLE: the hole is an ellipsoid
  // POLY: the corners at the first and last point (-1: none), the unit
  // tangents of the first and last segments and (3D) the patches beside it;
  // PCORNER: the volume's normal and (3D) the patches its curves lie beside
  int end[2] = {-1, -1}, pat[2] = {-1, -1};
  double t_first[3] = {0.0, 0.0, 0.0}, t_last[3] = {0.0, 0.0, 0.0}, n_vol[3] = {0.0, 0.0, 0.0};
  unsigned long long pmask = 0ull;
};

std::vector<HFeat> make_features(int D, int nh, int domain) {
  std::vector<HFeat> F;
  F.push_back({T_V, D, K_VOL});
  if (domain == SPH_DOMAIN_BALL) {   // the volume and its sphere
    F.push_back({D == 2 ? T_C : T_S, D - 1, K_SHELL});
    return F;
  }
  if (domain == SPH_DOMAIN_LEVEL_SET) {   // the volume and the zero level set
    F.push_back({D == 2 ? T_C : T_S, D - 1, K_LEVEL});
    return F;
  }
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

// the features of a geometry, with the imported curves and corners of a
// level-set domain (and in 3D the surface patches the curves split its zero
// set into) and the constant data their normals need
std::vector<HFeat> make_features_of(const sph_geometry *g) {
  if (g->domain != SPH_DOMAIN_LEVEL_SET || g->n_curves <= 0)
    return make_features(g->dim, g->n_holes, g->domain);
  const int D = g->dim, np = D == 3 ? g->n_patches : 0;
  std::vector<HFeat> F;
  F.push_back({T_V, D, K_VOL});
  for (int p = 0; p < np; ++p) {   // patches: the zero set's projection and normal
    HFeat f{T_S, 2, K_LEVEL};
    f.hole = p;
    F.push_back(f);
  }
  auto tangent_of = [&](int k, double *t) {
    const double *p0 = g->curve_pts + 3 * k, *p1 = g->curve_pts + 3 * (k + 1);
    double e[3] = {0.0, 0.0, 0.0}, ss = 0.0;
    for (int a = 0; a < D; ++a) {
      e[a] = p1[a] - p0[a];
      ss += e[a] * e[a];
    }
    const double l = std::sqrt(ss);
    for (int a = 0; a < D; ++a) t[a] = e[a] / l;
  };
  const int c0 = 1 + np;   // the first curve's feature
  for (int c = 0; c < g->n_curves; ++c) {
    HFeat f{T_C, 1, K_POLY};
    f.hole = c;
    f.end[0] = g->curve_ends[2 * c];
    f.end[1] = g->curve_ends[2 * c + 1];
    if (np > 0) {
      f.pat[0] = g->curve_patches[2 * c];
      f.pat[1] = g->curve_patches[2 * c + 1];
    }
    tangent_of(g->curve_off[c], f.t_first);
    tangent_of(g->curve_off[c + 1] - 2, f.t_last);
    F.push_back(f);
  }
  // the level set's geometry on the host, for the normal at a 3D vertex
  Geom hg{};
  hg.dim = D;
  hg.phi = g->phi;
  for (int a = 0; a < 3; ++a) {
    hg.pn[a] = a < D ? g->phi_n[a] : 1;
    hg.plo[a] = g->phi_lo[a];
    hg.ps[a] = a < D ? (double)(g->phi_n[a] - 1) / (g->phi_hi[a] - g->phi_lo[a]) : 0.0;
  }
  for (int m = 0; m < g->n_corners; ++m) {
    HFeat f{T_SI, 0, K_PCORNER};
    f.hole = m;
    for (int c = 0; c < g->n_curves; ++c) {
      const HFeat &C = F[c0 + c];
      if (C.end[0] != m && C.end[1] != m) continue;
      for (int e = 0; e < 2; ++e)
        if (C.pat[e] >= 0) f.pmask |= 1ull << C.pat[e];
    }
    if (D == 3) {   // towards decreasing phi at the vertex
      double mv[3];
      ls_unit<3>(hg, g->corners + 3 * m, mv);
      for (int a = 0; a < 3; ++a) f.n_vol[a] = -mv[a];
    } else {   // the normalised sum of the right normals of the end segments
      double s0 = 0.0, s1 = 0.0;
      for (int c = 0; c < g->n_curves; ++c)
        for (int e = 0; e < 2; ++e) {
          if (F[c0 + c].end[e] != m) continue;
          const double *t = e == 0 ? F[c0 + c].t_first : F[c0 + c].t_last;
          s0 += t[1];   // the right normal (t1, -t0)
          s1 -= t[0];
        }
      const double l = std::sqrt(s0 * s0 + s1 * s1);
      if (l > 0.0) {
        f.n_vol[0] = s0 / l;
        f.n_vol[1] = s1 / l;
      }
    }
    F.push_back(f);
  }
  return F;
}

// does the lower-dimensional feature B lie on the boundary of feature A?
bool on_boundary_of(const HFeat &A, const HFeat &B) {
  if (B.k >= A.k) return false;
  if (A.kind == K_VOL) return true;
  if (A.kind == K_POLY) return B.kind == K_PCORNER && (A.end[0] == B.hole || A.end[1] == B.hole);
  if (A.kind == K_LEVEL) {   // a 3D patch: the curves beside it and their end vertices
    if (B.kind == K_POLY) return B.pat[0] == A.hole || B.pat[1] == A.hole;
    if (B.kind == K_PCORNER) return ((B.pmask >> A.hole) & 1ull) != 0;
    return false;
  }
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
      N.mode = B.ell ? 3 : 2;
      N.hole = B.hole;
    } else if (B.kind == K_SHELL) {
      N.mode = 4;   // radially out of the ball, stored per particle
    } else if (B.kind == K_LEVEL) {
      N.mode = 5;   // against the level set's gradient, stored per particle
    } else if (B.kind == K_POLY) {
      N.mode = 6;   // stored per particle: in 2D the closest segment's right
                    // normal, in 3D against the level set's gradient
    } else if (B.kind == K_PCORNER) {
      for (int a = 0; a < 3; ++a) N.n[a] = B.n_vol[a];
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
  } else if (A.kind == K_POLY) {   // along the end segment, away from the curve
    for (int a = 0; a < 3; ++a) N.n[a] = A.end[0] == B.hole ? -A.t_first[a] : A.t_last[a];
  } else if (A.kind == K_LEVEL) {   // a patch: depends on the pair, computed in the sweep
    N.mode = B.kind == K_POLY ? 7 : 8;
  }
  return N;
}

// Device memory: from the caller's allocator (for instance PyTorch's caching
// allocator) when the parameters give one, from hipMalloc / hipFree otherwise.
// Memory is only released after the stream that used it has drained.
struct DevAlloc {
  void *(*alloc)(size_t, void *) = nullptr;
  void (*release)(void *, void *) = nullptr;
  void *ctx = nullptr;
  hipError_t get(void **p, size_t b) const {
    if (alloc) {
      *p = alloc(b, ctx);
      return *p ? hipSuccess : hipErrorOutOfMemory;
    }
    return hipMalloc(p, b);
  }
  void put(void *p) const {
    if (!p) return;
    if (release)
      release(p, ctx);
    else
      (void)hipFree(p);
  }
};

template <typename T>
T *dalloc(const DevAlloc &mem, size_t count, std::vector<void *> &owned, size_t &bytes) {
  void *p = nullptr;
  size_t b = std::max<size_t>(count, 1) * sizeof(T);
  b = (b + 255) & ~size_t(255);
  if (mem.get(&p, b) != hipSuccess) return nullptr;
  owned.push_back(p);
  bytes += b;
  return (T *)p;
}

}  // namespace


// a hole with unequal semi-axes (the first D of them) is an ellipsoid
static bool hole_is_ellipsoid(int D, const double *H) {
  return D == 2 ? H[4] != H[3] : (H[4] != H[3] || H[5] != H[3]);
}

static sph_status validate_geometry(const sph_geometry *g) {
  if (!g) return fail(SPH_ERR_INVALID_ARG, "null geometry");
  if (g->dim != 2 && g->dim != 3) return fail(SPH_ERR_INVALID_ARG, "dim must be 2 or 3");
  for (int a = 0; a < g->dim; ++a)
    if (!(g->lo[a] < g->hi[a]) || !std::isfinite(g->lo[a]) || !std::isfinite(g->hi[a]))
      return fail(SPH_ERR_INVALID_ARG, "empty or non-finite box on axis %d", a);
  if (g->n_holes < 0 || g->n_holes > MAXH)
    return fail(SPH_ERR_INVALID_ARG, "n_holes must be in [0, %d]", MAXH);
  if (g->n_holes > 0 && !g->holes) return fail(SPH_ERR_INVALID_ARG, "holes is NULL");
  for (int q = 0; q < g->n_holes; ++q) {
    const double *H = g->holes + 15 * q;
    double amax = 0.0;
    for (int a = 0; a < g->dim; ++a) {
      if (!(H[3 + a] > 0) || !std::isfinite(H[3 + a]))
        return fail(SPH_ERR_INVALID_ARG, "hole %d: semi-axes must be positive", q);
      amax = std::max(amax, H[3 + a]);
    }
    if (hole_is_ellipsoid(g->dim, H))   // the rotation must be orthonormal
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
          double t = 0.0;
          for (int m = 0; m < 3; ++m) t += H[6 + 3 * m + r] * H[6 + 3 * m + c];
          if (!(std::fabs(t - (r == c ? 1.0 : 0.0)) <= 1e-9))
            return fail(SPH_ERR_INVALID_ARG, "hole %d: rotation is not orthonormal", q);
        }
    for (int a = 0; a < g->dim; ++a)
      if (!(H[a] - amax > g->lo[a] && H[a] + amax < g->hi[a]))
        return fail(SPH_ERR_INVALID_ARG, "hole %d must lie strictly inside the box", q);
  }
  if (g->domain != SPH_DOMAIN_BOX && g->domain != SPH_DOMAIN_BALL &&
      g->domain != SPH_DOMAIN_LEVEL_SET)
    return fail(SPH_ERR_INVALID_ARG, "unknown domain kind");
  if (g->domain == SPH_DOMAIN_LEVEL_SET) {
    if (g->n_holes != 0) return fail(SPH_ERR_INVALID_ARG, "a level-set domain takes no holes");
    if (!g->phi) return fail(SPH_ERR_INVALID_ARG, "a level-set domain needs phi");
    int64_t nodes = 1;
    for (int a = 0; a < 3; ++a) {
      const int want = a < g->dim ? 2 : 1;
      if (g->phi_n[a] < want || g->phi_n[a] > 65536 || (a >= g->dim && g->phi_n[a] != 1))
        return fail(SPH_ERR_INVALID_ARG, "phi_n[%d] out of range", a);
      if (a < g->dim && !(g->phi_hi[a] > g->phi_lo[a] && std::isfinite(g->phi_lo[a]) &&
                          std::isfinite(g->phi_hi[a])))
        return fail(SPH_ERR_INVALID_ARG, "empty or non-finite level-set grid on axis %d", a);
      nodes *= g->phi_n[a];
    }
    if (nodes > (1ll << 27)) return fail(SPH_ERR_INVALID_ARG, "level-set grid has too many nodes");
    for (int64_t k = 0; k < nodes; ++k)
      if (!std::isfinite(g->phi[k])) return fail(SPH_ERR_INVALID_ARG, "phi is not finite");
    if (g->n_curves < 0 || g->n_corners < 0) return fail(SPH_ERR_INVALID_ARG, "negative curve count");
    if (g->n_curves > 0) {
      const int np = g->dim == 3 ? g->n_patches : 0;
      if (g->dim == 2 && g->n_patches != 0)
        return fail(SPH_ERR_INVALID_ARG, "n_patches must be 0 in 2D");
      if (g->dim == 3 && (g->n_patches < 1 || !g->curve_patches))
        return fail(SPH_ERR_INVALID_ARG, "3D imported curves need n_patches >= 1 and curve_patches");
      if (!g->curve_off || !g->curve_pts || !g->curve_ends || (g->n_corners > 0 && !g->corners))
        return fail(SPH_ERR_INVALID_ARG, "imported curves: NULL array");
      if (1 + np + g->n_curves + g->n_corners > MAXF)
        return fail(SPH_ERR_UNSUPPORTED, "too many imported features");
      if (g->curve_off[0] != 0) return fail(SPH_ERR_INVALID_ARG, "curve_off[0] must be 0");
      for (int c = 0; c < g->n_curves; ++c) {
        const int a0 = g->curve_off[c], a1 = g->curve_off[c + 1];
        if (a1 - a0 < 2 || a1 > (1 << 24))
          return fail(SPH_ERR_INVALID_ARG, "curve %d needs 2 to 2^24 points", c);
        for (int e = 0; e < 2; ++e) {
          if (g->curve_ends[2 * c + e] < -1 || g->curve_ends[2 * c + e] >= g->n_corners)
            return fail(SPH_ERR_INVALID_ARG, "curve %d: bad end corner", c);
          if (np > 0 && (g->curve_patches[2 * c + e] < -1 || g->curve_patches[2 * c + e] >= np))
            return fail(SPH_ERR_INVALID_ARG, "curve %d: bad patch", c);
        }
        for (int k = a0; k < a1; ++k) {
          const double *pt = g->curve_pts + 3 * k;
          for (int a = 0; a < g->dim; ++a)
            if (!std::isfinite(pt[a])) return fail(SPH_ERR_INVALID_ARG, "curve %d: non-finite point", c);
          if (k + 1 < a1 && pt[0] == pt[3] && pt[1] == pt[4] && (g->dim == 2 || pt[2] == pt[5]))
            return fail(SPH_ERR_INVALID_ARG, "curve %d: repeated point", c);
        }
      }
      for (int m = 0; m < 3 * g->n_corners; ++m)
        if (!std::isfinite(g->corners[m])) return fail(SPH_ERR_INVALID_ARG, "non-finite corner");
    }
  }
  if (g->domain == SPH_DOMAIN_BALL) {
    if (g->n_holes != 0) return fail(SPH_ERR_INVALID_ARG, "a ball domain takes no holes");
    const double e0 = g->hi[0] - g->lo[0];
    for (int a = 1; a < g->dim; ++a)
      if (!(std::fabs((g->hi[a] - g->lo[a]) - e0) <= 1e-12 * e0))
        return fail(SPH_ERR_INVALID_ARG, "a ball domain needs a cubic box");
  }
  return SPH_OK;
}

static sph_status validate(const sph_geometry *g, const sph_sizing *s, const sph_params *p) {
  if (!g || !s || !p) return fail(SPH_ERR_INVALID_ARG, "null geometry, sizing or params");
  if (sph_status st = validate_geometry(g)) return st;
  if (s->kind < 0 || s->kind > 4) return fail(SPH_ERR_INVALID_ARG, "unknown sizing kind");
  if (s->kind == 4) {
    if (!s->grid) return fail(SPH_ERR_INVALID_ARG, "gridded sizing needs a grid");
    int64_t nodes = 1;
    for (int a = 0; a < 3; ++a) {
      const int want = a < g->dim ? 2 : 1;
      if (s->grid_n[a] < want || s->grid_n[a] > 65536 || (a >= g->dim && s->grid_n[a] != 1))
        return fail(SPH_ERR_INVALID_ARG, "grid_n[%d] out of range", a);
      if (a < g->dim && !(s->grid_hi[a] > s->grid_lo[a] && std::isfinite(s->grid_lo[a]) &&
                          std::isfinite(s->grid_hi[a])))
        return fail(SPH_ERR_INVALID_ARG, "empty or non-finite grid box on axis %d", a);
      nodes *= s->grid_n[a];
    }
    if (nodes > (1ll << 27)) return fail(SPH_ERR_INVALID_ARG, "grid has too many nodes");
    for (int64_t k = 0; k < nodes; ++k)
      if (!(s->grid[k] > 0.0) || !std::isfinite(s->grid[k]))
        return fail(SPH_ERR_INVALID_ARG, "grid value %lld is not finite and positive", (long long)k);
  }
  if (s->kind == 3 && !std::isfinite(s->dcap))
    return fail(SPH_ERR_INVALID_ARG, "shell sizing needs a finite radius dcap");
  if (!(p->kernel_support == 0.0 || (p->kernel_support >= 1.0 && p->kernel_support <= 8.0)))
    return fail(SPH_ERR_INVALID_ARG, "kernel_support must be 0 or in [1, 8]");
  if (!(p->boundary_scale == 0.0 || (p->boundary_scale >= 0.25 && p->boundary_scale <= 8.0)))
    return fail(SPH_ERR_INVALID_ARG, "boundary_scale must be 0 or in [0.25, 8]");
  if (!(p->verlet_skin >= 0.0 && p->verlet_skin <= 2.0))
    return fail(SPH_ERR_INVALID_ARG, "verlet_skin must be in [0, 2]");
  if (p->cell_levels < 0 || p->cell_levels > MAXLEV)
    return fail(SPH_ERR_INVALID_ARG, "cell_levels must be in [0, %d]", MAXLEV);
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
  if (p->precision != SPH_FP64 && p->precision != SPH_FP32_MIXED &&
      p->precision != SPH_FP32_COMPENSATED)
    return fail(SPH_ERR_INVALID_ARG,
                "precision must be SPH_FP64, SPH_FP32_MIXED or SPH_FP32_COMPENSATED");
  if (p->max_neighbors < 0 || p->max_neighbors > 4096)
    return fail(SPH_ERR_INVALID_ARG, "max_neighbors must be in [0, 4096]");
  if (p->scan_tile != 0 && p->scan_tile != 2 && p->scan_tile != 4 && p->scan_tile != 8)
    return fail(SPH_ERR_INVALID_ARG, "scan_tile must be 0, 2, 4 or 8");
  if (!(p->cell_factor >= 0.0) || p->cell_factor > 16.0)
    return fail(SPH_ERR_INVALID_ARG, "cell_factor must be in [0, 16]");
  return SPH_OK;
}

// bounds of h_t over the box (points outside every hole), and its Lipschitz constant
static void sizing_bounds(const sph_geometry *g, const sph_sizing *s, double &hmin, double &hmax,
                          double &lip) {
  const int D = g->dim;
  auto corner = [&](int c, int a) { return ((c >> a) & 1) ? g->hi[a] : g->lo[a]; };
  hmin = s->h0;
  if (s->kind == 4) {
    // the multilinear interpolant stays within the node values; its slope
    // along axis a is a weighted mean of node differences along a
    const int n[3] = {s->grid_n[0], s->grid_n[1], D == 3 ? s->grid_n[2] : 1};
    const int64_t nodes = (int64_t)n[0] * n[1] * n[2];
    hmin = hmax = s->grid[0];
    for (int64_t k = 0; k < nodes; ++k) {
      hmin = std::min(hmin, s->grid[k]);
      hmax = std::max(hmax, s->grid[k]);
    }
    double sum = 0.0;
    for (int a = 0; a < D; ++a) {
      const int64_t st = a == 0 ? 1 : (a == 1 ? n[0] : (int64_t)n[0] * n[1]);
      double m = 0.0;
      for (int k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
          for (int i = 0; i < n[0]; ++i) {
            const int id[3] = {i, j, k};
            if (id[a] + 1 >= n[a]) continue;
            const int64_t q = ((int64_t)k * n[1] + j) * n[0] + i;
            m = std::max(m, std::fabs(s->grid[q + st] - s->grid[q]));
          }
      const double gr = m * (double)(n[a] - 1) / (s->grid_hi[a] - s->grid_lo[a]);
      sum += gr * gr;
    }
    lip = std::sqrt(sum);
    return;
  }
  if (s->kind == 0) {
    hmax = s->h0;
    lip = 0.0;
    return;
  }
  if (s->kind == 1 || s->kind == 3) {
    double far = 0.0;
    for (int c = 0; c < (1 << D); ++c) {
      double d2 = 0.0;
      for (int a = 0; a < D; ++a) d2 += (corner(c, a) - s->point[a]) * (corner(c, a) - s->point[a]);
      far = std::max(far, std::sqrt(d2));
    }
    // the farthest point of the box from `point` bounds | |x - point| - dcap |
    // by max(far - dcap, dcap)
    hmax = s->h0 + s->grad * (s->kind == 1 ? far : std::max(far - s->dcap, s->dcap));
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
    double amin = H[3];
    for (int a = 1; a < D; ++a) amin = std::min(amin, H[3 + a]);
    dmax = std::min(dmax, far - amin);
  }
  hmax = s->h0 * (1.0 + s->grad * dmax);
  lip = s->h0 * s->grad;
}



// copy a device column (slot order) to a host vector, ordered after the work
// already queued on the batch's stream
template <typename T>
static hipError_t pull(std::vector<T> &h, const void *d, size_t count, hipStream_t st) {
  h.resize(count);
  if (!count) return hipSuccess;
  hipError_t e = hipMemcpyAsync(h.data(), d, count * sizeof(T), hipMemcpyDeviceToHost, st);
  return e == hipSuccess ? hipStreamSynchronize(st) : e;
}

// ---------------------------------------------------------------------------
// a batch: resident jobs sharing one set of device arrays and one launch
// sequence per step
// ---------------------------------------------------------------------------
struct HostJob {
  bool live = false;
  int n = 0;
  double *d_grid = nullptr;   // gridded sizing: the job's copy of the node values
  double *d_phi = nullptr;    // level-set domain: the job's copy of phi
  double *d_cpts = nullptr;   // imported curves: the job's copy of their points
  int32_t *d_coff = nullptr;  // ... and of their offsets
  uint32_t ncell = 0, cbase = 0;
  int nf = 0;
  std::vector<HFeat> feats;
  JobDev dev{};
};

struct sph_batch {
  int D = 2, prec = SPH_FP64, cap = 64, tile = 4;
  bool use_graph = false, debug = false;
  int ncap = 0, jcap = 0;
  uint32_t ccap = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<void *> owned;
  size_t bytes = 0;
  DevAlloc mem;
  Parts P[2]{};
  int cur = 0;
  uint32_t *cell = nullptr, *rank = nullptr, *psrc = nullptr, *pkey = nullptr;
  uint32_t *cnt = nullptr, *cstart = nullptr, *ticket = nullptr;
  unsigned long long *scan_status = nullptr;
  uint32_t *nbr = nullptr, *nnb = nullptr;
  // Verlet candidate lists (skin > 0): lists, counts, x and h at the build,
  // displacement stripes and the rebuild flag
  double skin = 0.0;
  int skin_cap = 0;
  uint32_t *skin_list = nullptr, *nsk = nullptr;
  double4 *xref = nullptr;
  unsigned long long *vstate = nullptr;
  void *ap = nullptr, *acc = nullptr, *mid = nullptr;              // {ax, ay, az, 0} in the sweep precision
  double4 *enrm = nullptr;   // boundary normals of particles on holes (cell order)
  double *dbg_gam = nullptr, *dbg_vt = nullptr;
  double4 *dbg_vm = nullptr;
  JobDev *d_jobs = nullptr;
  Feat *d_feat = nullptr;
  unsigned long long *d_bmask = nullptr;
  BNorm *d_bn = nullptr;
  Group *d_grp = nullptr;
  JobStat *d_st = nullptr;
  unsigned int *d_gflags = nullptr;
  unsigned long long *smin = nullptr, *ssum = nullptr, *scnt = nullptr, *sesc = nullptr;
  std::vector<HostJob> jobs;
  int n = 0, njobs = 0;
  uint32_t ncell = 0;
  // captured step graphs: GRAPH_LONG steps and 2 steps (both start and end at
  // buffer parity 0); long runs replay the long one, so the gap the runtime
  // leaves between two graph launches comes once per GRAPH_LONG steps
  static constexpr int GRAPH_LONG = 16;
  hipGraphExec_t gexec = nullptr, gexec_long = nullptr;
  // profiling
  bool profiling = false;
  struct Ev {
    int kid;
    hipEvent_t a, b;
  };
  std::vector<Ev> ev_live;
  std::vector<hipEvent_t> ev_pool;
  double kms[KID_COUNT] = {};
  long long kcount[KID_COUNT] = {};

  ~sph_batch() {
    if (stream) (void)hipStreamSynchronize(stream);
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (gexec_long) (void)hipGraphExecDestroy(gexec_long);
    for (auto &e : ev_live) {
      (void)hipEventDestroy(e.a);
      (void)hipEventDestroy(e.b);
    }
    for (auto e : ev_pool) (void)hipEventDestroy(e);
    for (HostJob &J : jobs) {
      mem.put(J.d_grid);
      mem.put(J.d_phi);
      mem.put(J.d_cpts);
      mem.put(J.d_coff);
    }
    for (void *p : owned) mem.put(p);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }

  Batch dev() const {
    Batch B;
    B.jobs = d_jobs;
    B.feat = d_feat;
    B.bmask = d_bmask;
    B.bn = d_bn;
    B.grp = d_grp;
    B.st = d_st;
    B.gflags = d_gflags;
    B.smin = smin;
    B.ssum = ssum;
    B.scnt = scnt;
    B.sesc = sesc;
    B.n = n;
    B.cap = cap;
    B.ncell = ncell;
    B.ntiles = ntiles();
    B.njobs = njobs;
    B.enrm = enrm;
    B.skin_on = skin > 0.0 ? 1 : 0;
    B.skin_cap = skin_cap;
    B.skin = skin_list;
    B.nsk = nsk;
    B.xref = xref;
    B.vstate = vstate;
    return B;
  }
  uint32_t ntiles() const { return (ncell + SCAN_TILE - 1) / SCAN_TILE; }
  unsigned blocks(size_t count) const { return (unsigned)((count + BLOCK - 1) / BLOCK); }
  unsigned blocks8(size_t count) const { return (blocks(count) + 7u) / 8u * 8u; }

  void invalidate_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (gexec_long) (void)hipGraphExecDestroy(gexec_long);
    gexec = gexec_long = nullptr;
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
    if (!profiling) {
      hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, stream, args...);
      return hipGetLastError();
    }
    // profiling: the start and stop events are recorded by the dispatch
    // itself, so their interval is the kernel's execution alone
    hipEvent_t a = get_event(), b = get_event();
    hipExtLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, stream, a, b, 0, args...);
    hipError_t e = hipGetLastError();
    ev_live.push_back({kid, a, b});
    return e;
  }

  // the next step re-sorts the particles and rebuilds the Verlet lists
  // (after any change of the particles made outside a step; never captured)
  sph_status force_rebuild() {
    static const unsigned long long one = 1ull;
    if (skin > 0.0)
      HIPCHK(hipMemcpyAsync(vstate + VS_REBUILD, &one, sizeof one, hipMemcpyHostToDevice, stream));
    return SPH_OK;
  }

  sph_status hash_range(int i0, int i1) {
    if (sph_status st = force_rebuild()) return st;
    if (i1 <= i0) return SPH_OK;
    if (D == 2)
      HIPCHK(launch(KID_HASH, k_hash<2>, blocks(i1 - i0), BLOCK, dev(), P[cur], i0, i1, cell, rank, cnt));
    else
      HIPCHK(launch(KID_HASH, k_hash<3>, blocks(i1 - i0), BLOCK, dev(), P[cur], i0, i1, cell, rank, cnt));
    return SPH_OK;
  }

  // counting sort of the current particles into (cell, caller id) order;
  // needs cell / rank / cnt of the current buffer, leaves cnt cleared
  sph_status enqueue_sort() {
    const Batch B = dev();
    const unsigned long long *vs = skin > 0.0 ? vstate : nullptr;
    HIPCHK(launch(KID_SCAN, k_scan, B.ntiles, BLOCK, (const uint32_t *)cnt, cstart, ncell,
                  scan_status, ticket, B.ntiles, d_gflags, vs));
    HIPCHK(launch(KID_SCATTER, k_scatter, blocks(n), BLOCK, n, (const uint32_t *)cell,
                  (const uint32_t *)rank, (const uint32_t *)cstart, (const uint32_t *)P[cur].oid,
                  psrc, pkey, scan_status, B.ntiles, ticket, vs));
    if (D == 2)
      HIPCHK(launch(KID_RANK_GATHER, k_rank_gather<2>, blocks(n), BLOCK, B, n, (const uint32_t *)psrc,
                    (const uint32_t *)pkey, (const uint32_t *)cell, (const uint32_t *)cstart, cnt,
                    P[cur], P[1 - cur]));
    else
      HIPCHK(launch(KID_RANK_GATHER, k_rank_gather<3>, blocks(n), BLOCK, B, n, (const uint32_t *)psrc,
                    (const uint32_t *)pkey, (const uint32_t *)cell, (const uint32_t *)cstart, cnt,
                    P[cur], P[1 - cur]));
    // with Verlet lists the particles stay in P[cur]: a rebuild sorts them
    // into P[1 - cur] and the list build copies them back
    if (skin <= 0.0) cur = 1 - cur;
    return SPH_OK;
  }

  template <int DD>
  sph_status enqueue_lists_only() {
    HIPCHK(launch(KID_NBR_LISTS, k_nbr_forces<DD, double, false, 4>, blocks8(n), BLOCK, dev(),
                  P[cur], (const uint32_t *)cstart, 1, nbr, nnb, (double4 *)nullptr,
                  (double *)nullptr, (double *)nullptr, P[cur]));
    return SPH_OK;
  }

  // the neighbour + sweep A kernel for the batch's scan tile; with Verlet
  // lists, their build (which returns at once unless a rebuild is due) and
  // the kernel that filters them
  template <int DD, typename R, bool CMP>
  hipError_t launch_nbr_forces(const Batch &B, const Parts &s) {
    using R4 = typename Vec4<R>::T;
    auto go = [&](int kid, auto kern) {
      return launch(kid, kern, blocks8(n), BLOCK, B, s, (const uint32_t *)cstart, 0, nbr, nnb,
                    (R4 *)ap, dbg_gam, dbg_vt, s);
    };
    if (skin > 0.0) {
      // the build reads the particles a rebuild has just sorted into the
      // other buffer and copies them back into s
      const Parts &t = P[1 - cur];
      auto build = [&](auto kern) {
        return launch(KID_SKIN, kern, blocks8(n), BLOCK, B, t, (const uint32_t *)cstart, 0, nbr,
                      nnb, (R4 *)ap, dbg_gam, dbg_vt, s);
      };
      hipError_t e = tile == 2   ? build(k_nbr_forces<DD, R, false, 2, CMP, 1>)
                     : tile == 8 ? build(k_nbr_forces<DD, R, false, 8, CMP, 1>)
                                 : build(k_nbr_forces<DD, R, false, 4, CMP, 1>);
      if (e != hipSuccess) return e;
      // 3D: two lanes per particle (the tile sets only the build's batch)
      if constexpr (sizeof(R) == 4 && DD == 3 && SPH_VERLET_LANES == 2) {
        return launch(KID_NBR_FORCES, k_nbr_forces<DD, R, true, 4, CMP, 2, 2>, blocks8(2 * (size_t)n),
                      BLOCK, B, s, (const uint32_t *)cstart, 0, nbr, nnb, (R4 *)ap, dbg_gam, dbg_vt, s);
      }
      if (tile == 2) return go(KID_NBR_FORCES, k_nbr_forces<DD, R, true, 2, CMP, 2>);
      if (tile == 8) return go(KID_NBR_FORCES, k_nbr_forces<DD, R, true, 8, CMP, 2>);
      return go(KID_NBR_FORCES, k_nbr_forces<DD, R, true, 4, CMP, 2>);
    }
    if (tile == 2) return go(KID_NBR_FORCES, k_nbr_forces<DD, R, true, 2, CMP>);
    if (tile == 8) return go(KID_NBR_FORCES, k_nbr_forces<DD, R, true, 8, CMP>);
    return go(KID_NBR_FORCES, k_nbr_forces<DD, R, true, 4, CMP>);
  }

  template <int DD, typename R, bool CMP = false>
  sph_status enqueue_forces() {
    using R4 = typename Vec4<R>::T;
    const Batch B = dev();
    const Parts &s = P[cur];
    const unsigned gslots = (unsigned)((njobs * MAXF + BLOCK / 64 - 1) / (BLOCK / 64));
    HIPCHK((launch_nbr_forces<DD, R, CMP>(B, s)));
    HIPCHK(launch(KID_REDUCE_A, k_group_reduce, gslots, BLOCK, B, 0));
    if (DD == 3)   // 3D sweep B gathers precomputed mid-point records
      HIPCHK(launch(KID_MIDPOINT, k_midpoint<DD, R>, blocks(n), BLOCK, B, s, (const R4 *)ap,
                    (R4 *)mid));
    if (DD == 3 && SPH_SWEEPB_LANES == 2)   // 3D: two lanes per particle
      HIPCHK(launch(KID_SWEEP_B, k_sweep_b<DD, R, CMP, 2>, blocks8(2 * (size_t)n), BLOCK, B, s,
                    (const uint32_t *)nbr, (const uint32_t *)nnb, (const R4 *)ap, (const R4 *)mid,
                    (R4 *)acc, dbg_vm));
    else
      HIPCHK(launch(KID_SWEEP_B, k_sweep_b<DD, R, CMP>, blocks8(n), BLOCK, B, s, (const uint32_t *)nbr,
                    (const uint32_t *)nnb, (const R4 *)ap, (const R4 *)mid, (R4 *)acc, dbg_vm));
    HIPCHK(launch(KID_REDUCE_B, k_group_reduce, gslots, BLOCK, B, 1));
    HIPCHK(launch(KID_INTEGRATE_HASH, k_integrate_hash<DD, R>, blocks(n), BLOCK, B, s,
                  (const R4 *)acc, cell, rank, cnt));
    HIPCHK(launch(KID_CONTROL, k_control, 1u, BLOCK, B));
    return SPH_OK;
  }

  sph_status enqueue_step() {
    if (n == 0) return SPH_OK;
    if (sph_status st = enqueue_sort()) return st;
    if (D == 2)
      return prec == SPH_FP64 ? enqueue_forces<2, double>()
             : prec == SPH_FP32_COMPENSATED ? enqueue_forces<2, float, true>()
                                            : enqueue_forces<2, float>();
    return prec == SPH_FP64 ? enqueue_forces<3, double>()
           : prec == SPH_FP32_COMPENSATED ? enqueue_forces<3, float, true>()
                                          : enqueue_forces<3, float>();
  }

  // capture `steps` (even) steps into *out, unless already captured
  sph_status build_graph(hipGraphExec_t *out, int steps) {
    if (*out) return SPH_OK;
    const int saved = cur;
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
    sph_status st = SPH_OK;
    for (int k = 0; k < steps && !st; ++k) st = enqueue_step();
    hipError_t e = hipStreamEndCapture(stream, &graph);
    cur = saved;
    if (st) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    if (e != hipSuccess) return fail(SPH_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      *out = nullptr;
      return fail(SPH_ERR_DEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
    }
    return SPH_OK;
  }

  sph_status step(int n_steps) {
    int left = n_steps;
    if (n == 0) return SPH_OK;
    if (use_graph && !profiling) {
      // graphs are captured at buffer parity 0 (steps with Verlet lists keep
      // the parity, so any parity will do for them)
      if (left > 0 && cur != 0 && skin <= 0.0) {
        if (sph_status st = enqueue_step()) return st;
        --left;
      }
      if (left >= 2) {
        // both graphs are captured on first use, so that a later, longer
        // call does not capture inside its run
        if (sph_status st = build_graph(&gexec, 2)) return st;
        if (sph_status st = build_graph(&gexec_long, GRAPH_LONG)) return st;
        for (; left >= GRAPH_LONG; left -= GRAPH_LONG) HIPCHK(hipGraphLaunch(gexec_long, stream));
        for (; left >= 2; left -= 2) HIPCHK(hipGraphLaunch(gexec, stream));
      }
    }
    for (; left > 0; --left)
      if (sph_status st = enqueue_step()) return st;
    return SPH_OK;
  }

  // first slot of job j in the particle order (jobs are ordered by cell base)
  int job_first(int j) const {
    int first = 0;
    for (int k = 0; k < njobs; ++k)
      if (jobs[k].live && k != j && jobs[k].cbase < jobs[j].cbase) first += jobs[k].n;
    return first;
  }

  sph_status check_job(int j) {
    JobStat s{};
    unsigned int gf = 0;
    HIPCHK(hipMemcpyAsync(&s, d_st + j, sizeof s, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipMemcpyAsync(&gf, d_gflags, sizeof gf, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    if (gf) return fail(SPH_ERR_DEVICE, "cell-count scan lost a tile");
    if (s.nan_flag) return fail(SPH_ERR_STATE, "non-finite position of particle %u", s.nan_oid);
    if (s.overflow)
      return fail(SPH_ERR_STATE, "neighbour list overflow: %u neighbours > capacity %d "
                                 "(raise max_neighbors)", s.overflow_max, cap);
    if (s.skin_overflow)
      return fail(SPH_ERR_STATE, "Verlet list overflow: %u candidates > capacity %d "
                                 "(raise max_neighbors or lower verlet_skin)", s.skin_max, skin_cap);
    return SPH_OK;
  }

  bool valid_job(int j) const { return j >= 0 && j < njobs && jobs[j].live; }
};

#include "sph_setup.h"
#include "sph_tags.h"

// ---------------------------------------------------------------------------
// job description -> host job record
// ---------------------------------------------------------------------------
// Number of cell levels of a job: one per factor 2 of h when h spans more
// than a factor 4 (cell_levels = 0), capped by cell_levels and MAXLEV.
static int level_count(double hmin, double hmax, int want) {
  if (want == 1 || !(hmax > 4.0 * hmin)) return 1;
  int nl = (int)std::ceil(std::log2(hmax / hmin));
  return std::max(1, std::min(nl, want > 0 ? want : MAXLEV));
}

// cut-off radius r_c in units of h (sec. 2.3 gives no value); 0 selects 2,
// the kernel support at smoothing length h
static double support_of(const sph_params *p) {
  return p->kernel_support > 0.0 ? p->kernel_support : 2.0;
}

static void grid_of(const sph_geometry *g, const sph_sizing *s, const sph_params *p, Grid &Gr) {
  const int D = g->dim;
  double hmin, hmax, lip;
  sizing_bounds(g, s, hmin, hmax, lip);
  const double c = support_of(p);
  const double cf = p->cell_factor > 0 ? p->cell_factor : 1.0;
  const int nlev = level_count(hmin, hmax, p->cell_levels);
  // level l: h in [hmin 2^l, hmin 2^(l+1)), cell side c hmin 2^l cell_factor
  // (c hmin 2^l is the support radius of the level's smallest h)
  double scale = 1.0;
  auto cells_at = [&](int l, int a) {
    const double side = c * std::ldexp(hmin, l) * cf * scale;
    return std::max(1.0, std::floor((g->hi[a] - g->lo[a]) / side));
  };
  // cells of a level, with the padding of tiled rows (sph_device.h)
  auto level_cells = [&](double n0, double n1, double n2) {
    const int nn[3] = {(int)n0, (int)n1, (int)n2};
    if (rows_tiled(D, nn)) return n0 * (std::ceil(n1 / 8.0) * 8.0) * (std::ceil(n2 / 8.0) * 8.0);
    return n0 * n1 * n2;
  };
  for (;;) {
    double cells = 0.0;
    for (int l = 0; l < nlev; ++l)
      cells += level_cells(cells_at(l, 0), cells_at(l, 1), D == 3 ? cells_at(l, 2) : 1.0);
    if (cells <= 512.0 * 1024 * 1024) break;   // at most 2^29 cells per job
    scale *= 1.25;
  }
  std::memset(&Gr, 0, sizeof Gr);
  Gr.nlev = nlev;
  for (int a = 0; a < 3; ++a) Gr.lo[a] = g->lo[a];
  uint32_t total = 0;
  for (int l = 0; l < nlev; ++l) {
    Gr.lbase[l] = total;
    for (int a = 0; a < 3; ++a) {
      if (a < D) {
        Gr.nc[l][a] = (int)cells_at(l, a);
        Gr.inv_c[l][a] = Gr.nc[l][a] / (g->hi[a] - g->lo[a]);
        Gr.c[l][a] = (g->hi[a] - g->lo[a]) / Gr.nc[l][a];
        Gr.cmax = std::max(Gr.cmax, Gr.c[l][a]);
      } else {
        Gr.nc[l][a] = 1;
      }
    }
    total += (uint32_t)level_cells(Gr.nc[l][0], Gr.nc[l][1], Gr.nc[l][2]);
    Gr.hthr[l] = l == 0 ? 0.0 : std::ldexp(hmin, l);
    Gr.hcap[l] = l + 1 < nlev ? std::ldexp(hmin, l + 1) : hmax;
  }
  Gr.ncell = total;
  Gr.rmax = c * hmax * (1.0 + 1e-9);
  Gr.rfac = c * lip < 0.9 ? c * (1.0 + 1e-9) / (1.0 - c * lip) : 1e300;
  Gr.lip = lip;
}

static void fill_job(HostJob &J, const sph_geometry *g, const sph_sizing *s, const sph_params *p,
                     uint32_t cbase, int n) {
  const int D = g->dim;
  J.feats = make_features_of(g);
  for (HFeat &F : J.feats)
    if (F.kind == K_HOLE) F.ell = hole_is_ellipsoid(D, g->holes + 15 * F.hole) ? 1 : 0;
  J.nf = (int)J.feats.size();
  J.n = n;
  JobDev &d = J.dev;
  std::memset(&d, 0, sizeof d);
  Geom &G = d.g;
  G.dim = D;
  G.nf = J.nf;
  G.nh = g->n_holes;
  G.hkind = s->kind;
  G.domain = g->domain;
  if (g->domain == SPH_DOMAIN_BALL) {
    for (int a = 0; a < D; ++a) G.dc[a] = 0.5 * (g->lo[a] + g->hi[a]);
    G.dR = 0.5 * (g->hi[0] - g->lo[0]);
  }
  if (g->domain == SPH_DOMAIN_LEVEL_SET)
    for (int a = 0; a < 3; ++a) {
      G.pn[a] = a < D ? g->phi_n[a] : 1;
      G.plo[a] = g->phi_lo[a];
      G.ps[a] = a < D ? (double)(g->phi_n[a] - 1) / (g->phi_hi[a] - g->phi_lo[a]) : 0.0;
    }
  for (int a = 0; a < 3; ++a) {
    G.lo[a] = g->lo[a];
    G.hi[a] = g->hi[a];
    G.hpt[a] = s->point[a];
  }
  for (int q = 0; q < g->n_holes; ++q) {
    const double *H = g->holes + 15 * q;
    for (int a = 0; a < 3; ++a) G.hc[q][a] = H[a];
    G.hr[q] = H[3];
    G.hell[q] = hole_is_ellipsoid(D, H) ? 1 : 0;
    G.hamax[q] = 0.0;
    G.hamin[q] = H[3];
    for (int a = 0; a < 3; ++a) {
      G.ha[q][a] = H[3 + a];
      if (a < D) G.hamax[q] = std::max(G.hamax[q], H[3 + a]);
      if (a < D) G.hamin[q] = std::min(G.hamin[q], H[3 + a]);
    }
    for (int e = 0; e < 9; ++e) G.hR[q][e] = H[6 + e];
  }
  G.h0 = s->h0;
  G.grad = s->grad;
  G.dcap = s->dcap;
  if (s->kind == 4)
    for (int a = 0; a < 3; ++a) {
      G.gn[a] = a < D ? s->grid_n[a] : 1;
      G.glo[a] = s->grid_lo[a];
      G.gs[a] = a < D ? (double)(s->grid_n[a] - 1) / (s->grid_hi[a] - s->grid_lo[a]) : 0.0;
    }
  grid_of(g, s, p, d.G);
  d.ksup = support_of(p);
  d.klen = 0.5 * d.ksup;
  d.ksup2 = d.ksup * d.ksup;
  d.iband = 1.0 / (2.0 * d.klen * s->h0);   // J.g.h0
  d.bscale = p->boundary_scale > 0.0 ? p->boundary_scale : 1.0;
  d.G.cbase = cbase;
  J.ncell = d.G.ncell;
  J.cbase = cbase;
  Ctl &C = d.ctl;
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
  d.p0 = p->p0;
  d.bw = p->boundary_weighting;
  d.nf = J.nf;
  d.live = 1;
  d.vol = -1;
  for (int f = 0; f < J.nf; ++f)
    if (J.feats[f].kind == K_VOL) {
      d.vol = f;
      break;
    }
}

// 64 / 160 at r_c = 2h, scaled by (2.5 / 2)^D for the default r_c = 2.5h
static int64_t default_cap(int D) { return D == 2 ? 104 : 320; }

// entries of a Verlet candidate list: the neighbour capacity scaled by the
// reach's volume ratio at r_c = 2h (the largest ratio over r_c >= 2h), in
// whole blocks
static int64_t skin_capacity(int64_t cap, int D, double skin) {
  const double r = (2.0 + skin) / 2.0;
  const double m = std::ceil((double)cap * (D == 2 ? r * r : r * r * r));
  return ((int64_t)m + LB - 1) / LB * LB;
}

// the Verlet list's reach and rebuild limit of a job (skin delta): a pair
// closer than c max(h_i, h_j) now was closer than (c + delta) max(h) at the
// build if every particle has moved at most eps h (h at the build), eps =
// delta / (c L + 2), since h is L-Lipschitz
static void set_skin(JobDev &d, double skin) {
  const double c = d.ksup, cs = c + skin, lip = d.G.lip;
  d.ksup_s = cs;
  d.rfac_s = cs * lip < 0.9 ? cs * (1.0 + 1e-9) / (1.0 - cs * lip) : 1e300;
  d.rmax_s = d.G.rmax / c * cs;
  d.move_eps = skin > 0.0 ? skin / (c * lip + 2.0) * (1.0 - 1e-6) : 0.0;
}

// particle arrays of a job: count, non-NULL arrays, finite coordinates,
// feature ids of the geometry
static sph_status check_particles(const sph_geometry *g, int64_t n, const double *xyz,
                                  const int32_t *feature) {
  if (n < 0 || n > 0x7ffffff0ll || (n > 0 && (!xyz || !feature)))
    return fail(SPH_ERR_INVALID_ARG, "bad particle count or NULL particle arrays");
  const int nf = (int)make_features_of(g).size();
  if (nf > MAXF) return fail(SPH_ERR_UNSUPPORTED, "too many features (%d > %d)", nf, MAXF);
  for (int64_t i = 0; i < n; ++i) {
    if (feature[i] < 0 || feature[i] >= nf)
      return fail(SPH_ERR_INVALID_ARG, "particle %lld: feature %d out of range [0, %d)",
                  (long long)i, feature[i], nf);
    for (int a = 0; a < g->dim; ++a) {
      const double x = xyz[3 * i + a], slack = 1e-9 * (g->hi[a] - g->lo[a]);
      if (!std::isfinite(x))
        return fail(SPH_ERR_INVALID_ARG, "particle %lld: non-finite coordinate", (long long)i);
      if (x < g->lo[a] - slack || x > g->hi[a] + slack)
        return fail(SPH_ERR_INVALID_ARG, "particle %lld lies outside the box", (long long)i);
    }
  }
  return SPH_OK;
}

extern "C" int64_t sph_batch_footprint(const sph_batch_params *bp) {
  if (!bp || (bp->dim != 2 && bp->dim != 3) || bp->max_particles < 0 || bp->max_cells < 1 ||
      bp->max_jobs < 1 || bp->max_jobs > MAXJ || bp->max_neighbors < 0)
    return -1;
  const int64_t N = bp->max_particles + 8, C = bp->max_cells;
  const int64_t cap = (bp->max_neighbors ? bp->max_neighbors + LB - 1 : default_cap(bp->dim)) / LB * LB;
  const int64_t r4 = bp->precision == SPH_FP64 ? 32 : 16;
  int64_t b = 2 * N * (32 + 32 + 2 + 4 + 16);        // particle records, double buffered
  b += 4 * N * 4;                                     // cell, rank, psrc, pkey
  b += C * 4 + (C + 1) * 4 + ((C + SCAN_TILE - 1) / SCAN_TILE) * 8;
  b += N * cap * 4 + N * 4;                           // neighbour list + counts
  b += (bp->dim == 3 ? 3 : 2) * N * r4;               // a^p, a (and 3D mid-point records)
  b += N * 32;                                        // normals of particles on holes
  if (bp->debug_fields) b += N * (8 + 8 + 32);
  const int64_t slots = (int64_t)bp->max_jobs * MAXF;
  b += bp->max_jobs * (int64_t)sizeof(JobDev) + slots * (int64_t)(sizeof(Feat) + 8 + sizeof(Group)) +
       slots * MAXF * (int64_t)sizeof(BNorm) + bp->max_jobs * (int64_t)sizeof(JobStat);
  b += 2 * slots * NSTRIPE * 8 + 2 * (int64_t)bp->max_jobs * NSTRIPE * 8;
  if (!(bp->verlet_skin >= 0.0 && bp->verlet_skin <= 2.0)) return -1;
  if (bp->verlet_skin > 0.0)   // candidate lists, counts, x at the build, flags
    b += N * skin_capacity(cap, bp->dim, bp->verlet_skin) * 4 + N * 4 + N * 32 +
         VS_WORDS * 8;
  return b;
}

extern "C" int64_t sph_job_cells(const sph_geometry *g, const sph_sizing *s, const sph_params *p) {
  if (validate(g, s, p)) return -1;
  Grid Gr;
  grid_of(g, s, p, Gr);
  return (int64_t)Gr.ncell;
}

extern "C" sph_status sph_batch_create(const sph_batch_params *bp, sph_batch **out) {
  if (!out) return fail(SPH_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (sph_batch_footprint(bp) < 0) return fail(SPH_ERR_INVALID_ARG, "bad batch parameters");
  if (bp->precision != SPH_FP64 && bp->precision != SPH_FP32_MIXED &&
      bp->precision != SPH_FP32_COMPENSATED)
    return fail(SPH_ERR_INVALID_ARG,
                "precision must be SPH_FP64, SPH_FP32_MIXED or SPH_FP32_COMPENSATED");
  if (bp->max_particles > 0x7ffffff0ll || bp->max_cells > 0x7ffffff0ll)
    return fail(SPH_ERR_UNSUPPORTED, "capacity above 2^31");
  if (bp->max_neighbors > 4096) return fail(SPH_ERR_INVALID_ARG, "max_neighbors above 4096");
  if (bp->scan_tile != 0 && bp->scan_tile != 2 && bp->scan_tile != 4 && bp->scan_tile != 8)
    return fail(SPH_ERR_INVALID_ARG, "scan_tile must be 0, 2, 4 or 8");
  if ((bp->dev_alloc == nullptr) != (bp->dev_free == nullptr))
    return fail(SPH_ERR_INVALID_ARG, "dev_alloc and dev_free must be given together");
  auto *B = new sph_batch();
  B->mem.alloc = bp->dev_alloc;
  B->mem.release = bp->dev_free;
  B->mem.ctx = bp->alloc_ctx;
  B->D = bp->dim;
  B->prec = bp->precision;
  // capacity in whole list blocks
  B->cap = (bp->max_neighbors ? (bp->max_neighbors + LB - 1) / LB * LB : (int)default_cap(bp->dim));
  B->tile = bp->scan_tile ? bp->scan_tile : 4;
  B->use_graph = bp->use_graph != 0;
  B->debug = bp->debug_fields != 0;
  B->ncap = (int)bp->max_particles;
  B->ccap = (uint32_t)bp->max_cells;
  B->jcap = bp->max_jobs;
  B->jobs.resize(B->jcap);
  if (bp->stream) {
    B->stream = (hipStream_t)bp->stream;
  } else {
    if (hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking) != hipSuccess) {
      delete B;
      return fail(SPH_ERR_DEVICE, "hipStreamCreate failed");
    }
    B->own_stream = true;
  }
  auto &ow = B->owned;
  size_t &by = B->bytes;
  const size_t N = (size_t)B->ncap, NPAD = N + 8, C = B->ccap;
  const size_t tiles = (C + SCAN_TILE - 1) / SCAN_TILE;
  const size_t slots = (size_t)B->jcap * MAXF;
  bool ok = true;
  for (int b = 0; b < 2; ++b) {   // records padded past capacity: unclamped batched loads
    B->P[b].xh = dalloc<double4>(B->mem, NPAD, ow, by);
    B->P[b].v = dalloc<double4>(B->mem, NPAD, ow, by);
    B->P[b].f = dalloc<uint16_t>(B->mem, NPAD, ow, by);
    B->P[b].oid = dalloc<uint32_t>(B->mem, NPAD, ow, by);
    B->P[b].xf = dalloc<float4>(B->mem, NPAD, ow, by);
    ok = ok && B->P[b].xh && B->P[b].v && B->P[b].f && B->P[b].oid && B->P[b].xf;
  }
  B->cell = dalloc<uint32_t>(B->mem, N, ow, by);
  B->rank = dalloc<uint32_t>(B->mem, N, ow, by);
  B->psrc = dalloc<uint32_t>(B->mem, N, ow, by);
  B->pkey = dalloc<uint32_t>(B->mem, N, ow, by);
  B->cnt = dalloc<uint32_t>(B->mem, C, ow, by);
  B->cstart = dalloc<uint32_t>(B->mem, C + 1, ow, by);
  B->scan_status = dalloc<unsigned long long>(B->mem, tiles, ow, by);
  B->ticket = dalloc<uint32_t>(B->mem, 1, ow, by);
  B->nbr = dalloc<uint32_t>(B->mem, N * (size_t)B->cap, ow, by);
  B->nnb = dalloc<uint32_t>(B->mem, N, ow, by);
  const size_t r4 = B->prec == SPH_FP64 ? sizeof(double4) : sizeof(float4);
  B->ap = dalloc<char>(B->mem, N * r4, ow, by);
  B->acc = dalloc<char>(B->mem, N * r4, ow, by);
  if (B->D == 3) B->mid = dalloc<char>(B->mem, N * r4, ow, by);   // mid-point records (3D sweep B)
  B->enrm = dalloc<double4>(B->mem, N, ow, by);
  B->skin = bp->verlet_skin;
  if (B->skin > 0.0) {
    B->skin_cap = (int)skin_capacity(B->cap, B->D, B->skin);
    B->skin_list = dalloc<uint32_t>(B->mem, N * (size_t)B->skin_cap, ow, by);
    B->nsk = dalloc<uint32_t>(B->mem, N, ow, by);
    B->xref = dalloc<double4>(B->mem, N, ow, by);
    B->vstate = dalloc<unsigned long long>(B->mem, VS_WORDS, ow, by);
    ok = ok && B->skin_list && B->nsk && B->xref && B->vstate;
  }
  if (B->debug) {
    B->dbg_gam = dalloc<double>(B->mem, N, ow, by);
    B->dbg_vt = dalloc<double>(B->mem, N, ow, by);
    B->dbg_vm = dalloc<double4>(B->mem, N, ow, by);
    ok = ok && B->dbg_gam && B->dbg_vt && B->dbg_vm;
  }
  B->d_jobs = dalloc<JobDev>(B->mem, B->jcap, ow, by);
  B->d_feat = dalloc<Feat>(B->mem, slots, ow, by);
  B->d_bmask = dalloc<unsigned long long>(B->mem, slots, ow, by);
  B->d_bn = dalloc<BNorm>(B->mem, slots * MAXF, ow, by);
  B->d_grp = dalloc<Group>(B->mem, slots, ow, by);
  B->d_st = dalloc<JobStat>(B->mem, B->jcap, ow, by);
  B->d_gflags = dalloc<unsigned int>(B->mem, 4, ow, by);
  B->smin = dalloc<unsigned long long>(B->mem, slots * NSTRIPE, ow, by);
  B->ssum = dalloc<unsigned long long>(B->mem, slots * NSTRIPE, ow, by);
  B->scnt = dalloc<unsigned long long>(B->mem, (size_t)B->jcap * NSTRIPE, ow, by);
  B->sesc = dalloc<unsigned long long>(B->mem, (size_t)B->jcap * NSTRIPE, ow, by);
  ok = ok && B->cell && B->rank && B->psrc && B->pkey && B->cnt && B->cstart && B->scan_status &&
       B->ticket && B->nbr && B->nnb && B->ap && B->acc && (B->mid || B->D == 2) && B->enrm && B->d_jobs && B->d_feat && B->d_bmask &&
       B->d_bn && B->d_grp && B->d_st && B->d_gflags && B->smin && B->ssum && B->scnt && B->sesc;
  if (!ok) {
    delete B;
    return fail(SPH_ERR_OUT_OF_MEMORY, "device allocation of %zu bytes failed", by);
  }
  hipError_t e = hipMemset(B->cnt, 0, sizeof(uint32_t) * C);
  if (e == hipSuccess) e = hipMemset(B->scan_status, 0, 8 * std::max<size_t>(tiles, 1));
  if (e == hipSuccess) e = hipMemset(B->ticket, 0, 4);
  if (e == hipSuccess) e = hipMemset(B->nnb, 0, 4 * std::max<size_t>(N, 1));
  if (e == hipSuccess) e = hipMemset(B->d_grp, 0, sizeof(Group) * slots);
  if (e == hipSuccess) e = hipMemset(B->d_st, 0, sizeof(JobStat) * B->jcap);
  if (e == hipSuccess) e = hipMemset(B->d_gflags, 0, 16);
  if (e == hipSuccess) e = hipMemset(B->smin, 0xff, 8 * slots * NSTRIPE);   // minimum identity
  if (e == hipSuccess) e = hipMemset(B->ssum, 0, 8 * slots * NSTRIPE);
  if (e == hipSuccess) e = hipMemset(B->scnt, 0, 8 * (size_t)B->jcap * NSTRIPE);
  if (e == hipSuccess) e = hipMemset(B->sesc, 0, 8 * (size_t)B->jcap * NSTRIPE);
  if (e == hipSuccess) e = hipMemset(B->P[0].f, 0, 2 * NPAD);
  if (e == hipSuccess) e = hipMemset(B->P[1].f, 0, 2 * NPAD);
  if (e == hipSuccess) e = hipMemset(B->P[0].xf, 0, sizeof(float4) * NPAD);
  if (e == hipSuccess) e = hipMemset(B->P[1].xf, 0, sizeof(float4) * NPAD);
  if (e == hipSuccess && B->skin > 0.0) {
    e = hipMemset(B->vstate, 0, 8 * VS_WORDS);
    if (e == hipSuccess) e = hipMemset(B->nsk, 0, 4 * std::max<size_t>(N, 1));
    if (e == hipSuccess) e = hipMemset(B->xref, 0, sizeof(double4) * std::max<size_t>(N, 1));
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    delete B;
    return fail(SPH_ERR_DEVICE, "batch initialisation failed: %s", hipGetErrorString(e));
  }
  *out = B;
  return SPH_OK;
}

extern "C" void sph_batch_destroy(sph_batch *b) { delete b; }

extern "C" sph_status sph_batch_add(sph_batch *b, const sph_geometry *g, const sph_sizing *s,
                                    const sph_params *p, int64_t n, const double *xyz,
                                    const int32_t *feature, int32_t *job) {
  if (!b) return fail(SPH_ERR_INVALID_ARG, "null batch");
  if (sph_status st = validate(g, s, p)) return st;
  if (g->dim != b->D) return fail(SPH_ERR_INVALID_ARG, "job dimension %d != batch dimension %d",
                                  g->dim, b->D);
  if (sph_status st = check_particles(g, n, xyz, feature)) return st;
  const int nf = (int)make_features_of(g).size();
  int slot = -1;
  for (int j = 0; j < b->jcap; ++j)
    if (!b->jobs[j].live) {
      slot = j;
      break;
    }
  if (slot < 0) return fail(SPH_ERR_OUT_OF_MEMORY, "no free job slot (max_jobs %d)", b->jcap);
  HostJob J;
  fill_job(J, g, s, p, b->ncell, (int)n);
  set_skin(J.dev, b->skin);
  if ((int64_t)b->n + n > b->ncap)
    return fail(SPH_ERR_OUT_OF_MEMORY, "particle capacity %d exceeded", b->ncap);
  if ((uint64_t)b->ncell + J.ncell > b->ccap)
    return fail(SPH_ERR_OUT_OF_MEMORY, "cell capacity %u exceeded (job needs %u)", b->ccap, J.ncell);
  HIPCHK(hipStreamSynchronize(b->stream));
  if (s->kind == 4) {   // the job's own device copy of the sizing grid
    const size_t bytes = sizeof(double) * (size_t)s->grid_n[0] * s->grid_n[1] * s->grid_n[2];
    if (b->mem.get((void **)&J.d_grid, bytes) != hipSuccess)
      return fail(SPH_ERR_OUT_OF_MEMORY, "no device memory for the sizing grid");
    hipError_t ge = hipMemcpyAsync(J.d_grid, s->grid, bytes, hipMemcpyHostToDevice, b->stream);
    if (ge == hipSuccess) ge = hipStreamSynchronize(b->stream);
    if (ge != hipSuccess) {
      b->mem.put(J.d_grid);
      return fail(SPH_ERR_DEVICE, "sizing grid upload failed: %s", hipGetErrorString(ge));
    }
    J.dev.g.grid = J.d_grid;
  }
  if (g->domain == SPH_DOMAIN_LEVEL_SET) {   // the job's own device copy of phi
    const size_t bytes = sizeof(double) * (size_t)g->phi_n[0] * g->phi_n[1] * g->phi_n[2];
    hipError_t pe = b->mem.get((void **)&J.d_phi, bytes);
    if (pe == hipSuccess) pe = hipMemcpyAsync(J.d_phi, g->phi, bytes, hipMemcpyHostToDevice, b->stream);
    if (pe == hipSuccess) pe = hipStreamSynchronize(b->stream);
    if (pe != hipSuccess) {
      b->mem.put(J.d_phi);
      b->mem.put(J.d_grid);
      return fail(SPH_ERR_DEVICE, "level-set upload failed: %s", hipGetErrorString(pe));
    }
    J.dev.g.phi = J.d_phi;
  }
  if (g->domain == SPH_DOMAIN_LEVEL_SET && g->n_curves > 0) {   // imported curves
    const size_t np = (size_t)g->curve_off[g->n_curves];
    const size_t pb = sizeof(double) * 3 * np, ob = sizeof(int32_t) * (size_t)(g->n_curves + 1);
    hipError_t ce = b->mem.get((void **)&J.d_cpts, pb);
    if (ce == hipSuccess) ce = b->mem.get((void **)&J.d_coff, ob);
    if (ce == hipSuccess) ce = hipMemcpyAsync(J.d_cpts, g->curve_pts, pb, hipMemcpyHostToDevice, b->stream);
    if (ce == hipSuccess) ce = hipMemcpyAsync(J.d_coff, g->curve_off, ob, hipMemcpyHostToDevice, b->stream);
    if (ce == hipSuccess) ce = hipStreamSynchronize(b->stream);
    if (ce != hipSuccess) {
      for (void *buf : {(void *)J.d_cpts, (void *)J.d_coff, (void *)J.d_phi, (void *)J.d_grid})
        b->mem.put(buf);
      return fail(SPH_ERR_DEVICE, "curve upload failed: %s", hipGetErrorString(ce));
    }
    J.dev.g.cpts = J.d_cpts;
    J.dev.g.coff = J.d_coff;
  }
  const int D = b->D;
  // tables of the job's feature slots
  std::vector<Feat> hf(MAXF);
  std::vector<unsigned long long> hm(MAXF, 0ull);
  std::vector<BNorm> hb((size_t)MAXF * MAXF);
  std::memset(hf.data(), 0, sizeof(Feat) * MAXF);
  std::memset(hb.data(), 0, sizeof(BNorm) * MAXF * MAXF);
  for (int i = 0; i < nf; ++i) {
    const HFeat &F = J.feats[i];
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
      hb[(size_t)i * MAXF + j] = boundary_normal(D, F, J.feats[j]);
      if (i != j && on_boundary_of(F, J.feats[j])) hm[i] |= 1ull << j;
    }
  }
  std::vector<int64_t> counts(nf, 0);
  for (int64_t i = 0; i < n; ++i) counts[feature[i]]++;
  double hmin, hmax, lip;
  sizing_bounds(g, s, hmin, hmax, lip);
  std::vector<Group> hg(MAXF);
  for (int q = 0; q < MAXF; ++q) {
    Group &Q = hg[q];
    std::memset(&Q, 0, sizeof Q);
    if (q >= nf) continue;
    Q.tracked = J.feats[q].type != T_SI && counts[q] > 0;
    Q.active = Q.tracked;
    Q.phase = PH_ONE;
    Q.count = (int32_t)counts[q];
    Q.eps = p->eps_damp;
    Q.esys = HUGE_VAL;
    double db = p->dt_max;
    std::memcpy(&Q.dt1_bits, &db, 8);
    std::memcpy(&Q.dt_bits, &db, 8);
    // fixed-point scale of the V~ sum: V~_i <= h^k / alpha_k, keep the
    // feature's total below 2^62
    const int k = J.feats[q].k;
    const double alpha = k == 1 ? 0.625 : (k == 2 ? 7.0 / (4.0 * M_PI) : 21.0 / (16.0 * M_PI));
    double bound = (double)std::max<int64_t>(counts[q], 1) * std::pow(hmax, k) / alpha;
    int ex = 62 - (int)std::ceil(std::log2(bound * 2.0));
    Q.vscale = std::ldexp(1.0, std::min(ex, 1000));
  }
  // particle records appended after the resident jobs (their cells follow
  // every resident cell, so the order stays sorted by cell)
  const size_t N = (size_t)n;
  std::vector<double4> xh(N);
  std::vector<uint32_t> oid(N);
  std::vector<uint16_t> f16(N);
  for (size_t i = 0; i < N; ++i) {
    xh[i] = make_double4(xyz[3 * i], xyz[3 * i + 1], D == 3 ? xyz[3 * i + 2] : 0.0, 0.0);
    oid[i] = (uint32_t)i;
    f16[i] = (uint16_t)(slot * MAXF + feature[i]);
  }
  const Parts &P = b->P[b->cur];
  const size_t o = (size_t)b->n;
  JobStat js{};
  js.live = 1;
  hipError_t e = hipSuccess;
  // every upload and clear is queued on the batch's stream, in order with the
  // hash that follows (a null-stream copy or memset is not ordered with a
  // non-blocking stream); the host vectors live until the synchronisation
  hipStream_t q = b->stream;
  if (N) e = hipMemcpyAsync(P.xh + o, xh.data(), N * sizeof(double4), hipMemcpyHostToDevice, q);
  if (e == hipSuccess && N) e = hipMemsetAsync(P.v + o, 0, N * sizeof(double4), q);
  if (e == hipSuccess && N) e = hipMemcpyAsync(P.oid + o, oid.data(), N * 4, hipMemcpyHostToDevice, q);
  if (e == hipSuccess && N) e = hipMemcpyAsync(P.f + o, f16.data(), N * 2, hipMemcpyHostToDevice, q);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_feat + slot * MAXF, hf.data(), sizeof(Feat) * MAXF,
                       hipMemcpyHostToDevice, q);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_bmask + slot * MAXF, hm.data(), 8 * MAXF, hipMemcpyHostToDevice, q);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_bn + (size_t)slot * MAXF * MAXF, hb.data(),
                       sizeof(BNorm) * MAXF * MAXF, hipMemcpyHostToDevice, q);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_grp + slot * MAXF, hg.data(), sizeof(Group) * MAXF,
                       hipMemcpyHostToDevice, q);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_jobs + slot, &J.dev, sizeof(JobDev), hipMemcpyHostToDevice, q);
  if (e == hipSuccess) e = hipMemcpyAsync(b->d_st + slot, &js, sizeof js, hipMemcpyHostToDevice, q);
  if (e == hipSuccess && J.ncell) e = hipMemsetAsync(b->cnt + b->ncell, 0, 4 * (size_t)J.ncell, q);
  if (e == hipSuccess) e = hipStreamSynchronize(q);
  else (void)hipStreamSynchronize(q);
  if (e != hipSuccess) {
    for (void *buf : {(void *)J.d_cpts, (void *)J.d_coff, (void *)J.d_phi, (void *)J.d_grid})
      b->mem.put(buf);
    return fail(SPH_ERR_DEVICE, "job upload failed: %s", hipGetErrorString(e));
  }
  J.live = true;
  b->jobs[slot] = J;
  const int i0 = b->n;
  b->n += (int)n;
  b->ncell += J.ncell;
  b->njobs = std::max(b->njobs, slot + 1);
  b->invalidate_graph();
  if (sph_status st = b->hash_range(i0, b->n)) return st;
  HIPCHK(hipStreamSynchronize(b->stream));
  if (job) *job = slot;
  return SPH_OK;
}

extern "C" sph_status sph_batch_remove(sph_batch *b, int32_t job) {
  if (!b || !b->valid_job(job)) return fail(SPH_ERR_INVALID_ARG, "no such job");
  HIPCHK(hipStreamSynchronize(b->stream));
  // surviving jobs in their current (cell base) order, copied contiguously
  std::vector<int> order;
  for (int j = 0; j < b->njobs; ++j)
    if (b->jobs[j].live && j != job) order.push_back(j);
  std::sort(order.begin(), order.end(),
            [&](int x, int y) { return b->jobs[x].cbase < b->jobs[y].cbase; });
  const Parts &src = b->P[b->cur], &dst = b->P[1 - b->cur];
  size_t off = 0;
  uint32_t cb = 0;
  for (int j : order) {
    HostJob &J = b->jobs[j];
    const size_t first = (size_t)b->job_first(j), m = (size_t)J.n;
    if (m) {
      HIPCHK(hipMemcpyAsync(dst.xh + off, src.xh + first, m * sizeof(double4), hipMemcpyDeviceToDevice, b->stream));
      HIPCHK(hipMemcpyAsync(dst.v + off, src.v + first, m * sizeof(double4), hipMemcpyDeviceToDevice, b->stream));
      HIPCHK(hipMemcpyAsync(dst.f + off, src.f + first, m * 2, hipMemcpyDeviceToDevice, b->stream));
      HIPCHK(hipMemcpyAsync(dst.oid + off, src.oid + first, m * 4, hipMemcpyDeviceToDevice, b->stream));
    }
    off += m;
  }
  // new cell bases
  for (int j : order) {
    HostJob &J = b->jobs[j];
    J.cbase = cb;
    J.dev.G.cbase = cb;
    cb += J.ncell;
    HIPCHK(hipMemcpyAsync(b->d_jobs + j, &J.dev, sizeof(JobDev), hipMemcpyHostToDevice, b->stream));
  }
  HostJob &R = b->jobs[job];
  R.live = false;
  R.dev.live = 0;
  R.dev.g.grid = nullptr;
  R.dev.g.phi = nullptr;
  R.dev.g.cpts = nullptr;
  R.dev.g.coff = nullptr;
  HIPCHK(hipMemsetAsync(b->d_grp + job * MAXF, 0, sizeof(Group) * MAXF, b->stream));
  HIPCHK(hipMemsetAsync(b->d_st + job, 0, sizeof(JobStat), b->stream));
  HIPCHK(hipMemcpyAsync(b->d_jobs + job, &R.dev, sizeof(JobDev), hipMemcpyHostToDevice, b->stream));
  HIPCHK(hipMemsetAsync(b->cnt, 0, 4 * (size_t)std::max(b->ncell, 1u), b->stream));
  HIPCHK(hipStreamSynchronize(b->stream));
  // no kernel that reads them is queued any more
  b->mem.put(R.d_grid);
  b->mem.put(R.d_phi);
  b->mem.put(R.d_cpts);
  b->mem.put(R.d_coff);
  R.d_grid = nullptr;
  R.d_phi = nullptr;
  R.d_cpts = nullptr;
  R.d_coff = nullptr;
  b->cur = 1 - b->cur;
  b->n = (int)off;
  b->ncell = cb;
  while (b->njobs > 0 && !b->jobs[b->njobs - 1].live) b->njobs--;
  b->invalidate_graph();
  if (sph_status st = b->hash_range(0, b->n)) return st;
  HIPCHK(hipStreamSynchronize(b->stream));
  return SPH_OK;
}

extern "C" sph_status sph_batch_step(sph_batch *b, int32_t n_steps) {
  if (!b || n_steps < 0) return fail(SPH_ERR_INVALID_ARG, "bad batch or step count");
  return b->step(n_steps);
}

extern "C" sph_status sph_batch_sync(sph_batch *b) {
  if (!b) return fail(SPH_ERR_INVALID_ARG, "null batch");
  HIPCHK(hipStreamSynchronize(b->stream));
  return SPH_OK;
}

extern "C" sph_status sph_batch_status(sph_batch *b, int32_t *live, int32_t *converged,
                                       int64_t *steps, int32_t cap) {
  if (!b) return fail(SPH_ERR_INVALID_ARG, "null batch");
  HIPCHK(hipStreamSynchronize(b->stream));
  std::vector<JobStat> st(b->jcap);
  HIPCHK(hipMemcpyAsync(st.data(), b->d_st, sizeof(JobStat) * b->jcap, hipMemcpyDeviceToHost, b->stream));
  HIPCHK(hipStreamSynchronize(b->stream));
  for (int j = 0; j < cap; ++j) {
    const bool ok = j < b->jcap && b->jobs[j].live;
    if (live) live[j] = ok;
    if (converged) converged[j] = ok ? st[j].converged : 0;
    if (steps) steps[j] = ok ? (int64_t)st[j].steps : 0;
  }
  return SPH_OK;
}

extern "C" sph_status sph_batch_positions(sph_batch *b, int32_t job, double *xyz, int32_t *feature,
                                          int64_t capacity, int64_t *n_out) {
  if (!b || !b->valid_job(job)) return fail(SPH_ERR_INVALID_ARG, "no such job");
  const HostJob &J = b->jobs[job];
  if (n_out) *n_out = J.n;
  if (!xyz && !feature) return SPH_OK;
  if (capacity < J.n) return fail(SPH_ERR_INVALID_ARG, "capacity %lld < %d particles",
                                  (long long)capacity, J.n);
  HIPCHK(hipStreamSynchronize(b->stream));
  if (sph_status st = b->check_job(job)) return st;
  const Parts &s = b->P[b->cur];
  const size_t first = (size_t)b->job_first(job);
  std::vector<uint32_t> oid;
  HIPCHK(pull(oid, s.oid + first, J.n, b->stream));
  if (xyz) {
    std::vector<double4> xh;
    HIPCHK(pull(xh, s.xh + first, J.n, b->stream));
    for (int i = 0; i < J.n; ++i) {
      double *o = xyz + 3 * (size_t)oid[i];
      o[0] = xh[i].x;
      o[1] = xh[i].y;
      o[2] = b->D == 3 ? xh[i].z : 0.0;
    }
  }
  if (feature) {
    std::vector<uint16_t> f;
    HIPCHK(pull(f, s.f + first, J.n, b->stream));
    for (int i = 0; i < J.n; ++i) feature[oid[i]] = f[i] % MAXF;
  }
  return SPH_OK;
}

extern "C" sph_status sph_batch_error(sph_batch *b, int32_t job, double *e_sys, int32_t *phase,
                                      int32_t *converged, int64_t *step) {
  if (!b || !b->valid_job(job)) return fail(SPH_ERR_INVALID_ARG, "no such job");
  HIPCHK(hipStreamSynchronize(b->stream));
  if (sph_status st = b->check_job(job)) return st;
  std::vector<Group> G(MAXF);
  HIPCHK(hipMemcpyAsync(G.data(), b->d_grp + job * MAXF, sizeof(Group) * MAXF, hipMemcpyDeviceToHost, b->stream));
  HIPCHK(hipStreamSynchronize(b->stream));
  JobStat S;
  HIPCHK(hipMemcpyAsync(&S, b->d_st + job, sizeof S, hipMemcpyDeviceToHost, b->stream));
  HIPCHK(hipStreamSynchronize(b->stream));
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

extern "C" sph_status sph_batch_counters(sph_batch *b, int32_t job, double *out) {
  if (!b || !out || !b->valid_job(job)) return fail(SPH_ERR_INVALID_ARG, "bad argument");
  HIPCHK(hipStreamSynchronize(b->stream));
  JobStat S;
  HIPCHK(hipMemcpyAsync(&S, b->d_st + job, sizeof S, hipMemcpyDeviceToHost, b->stream));
  HIPCHK(hipStreamSynchronize(b->stream));
  out[0] = (double)S.steps;
  out[1] = (double)S.escaped;
  out[2] = (double)S.inter_total;
  out[3] = (double)S.inter_last;
  return SPH_OK;
}

// ---------------------------------------------------------------------------
// the single-job API: a batch holding one job (slot 0)
// ---------------------------------------------------------------------------
struct sph_mesh {
  sph_batch *b = nullptr;
  int job = 0;
  // set-up from the problem statement: the factor h was scaled by, and the
  // particles placed per feature
  double h_scale = 1.0;
  std::vector<int64_t> counts;
  ~sph_mesh() { delete b; }
};

extern "C" sph_status sph_mesh_create_with_particles(const sph_geometry *g, const sph_sizing *s,
                                                     const sph_params *p, int64_t n,
                                                     const double *xyz, const int32_t *feature,
                                                     sph_mesh **out) {
  if (!out) return fail(SPH_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (sph_status st = validate(g, s, p)) return st;
  if (sph_status st = check_particles(g, n, xyz, feature)) return st;
  sph_batch_params bp{};
  bp.dev_alloc = p->dev_alloc;
  bp.dev_free = p->dev_free;
  bp.alloc_ctx = p->alloc_ctx;
  bp.dim = g->dim;
  bp.precision = p->precision;
  bp.max_particles = std::max<int64_t>(n, 1);
  bp.max_cells = sph_job_cells(g, s, p);
  bp.max_jobs = 1;
  bp.max_neighbors = p->max_neighbors;
  bp.scan_tile = p->scan_tile;
  bp.use_graph = p->use_graph;
  bp.debug_fields = p->debug_fields;
  bp.stream = p->stream;
  bp.verlet_skin = p->verlet_skin;
  auto *M = new sph_mesh();
  if (sph_status st = sph_batch_create(&bp, &M->b)) {
    delete M;
    return st;
  }
  if (sph_status st = sph_batch_add(M->b, g, s, p, n, xyz, feature, &M->job)) {
    delete M;
    return st;
  }
  *out = M;
  return SPH_OK;
}

// Algorithm 1's set-up from the problem statement: feature masses and the
// particle split (sec. 3.2), h scaled to the budget (reading R25), and, when
// want_particles, the initial particles drawn from a Mersenne Twister
// (sec. 3.6).  Host work only.
static sph_status problem_setup(const sph_geometry *g, const sph_sizing *s, const sph_params *p,
                                bool want_particles, setup::Plan &P, sph_sizing &s2,
                                std::vector<double> &xyz, std::vector<int32_t> &feat) {
  if (sph_status st = validate(g, s, p)) return st;
  if (g->domain != SPH_DOMAIN_BOX && g->domain != SPH_DOMAIN_BALL)
    return fail(SPH_ERR_UNSUPPORTED, "set-up from the problem statement takes a box or ball "
                                     "domain; give a level-set domain's particles to "
                                     "sph_mesh_create_with_particles");
  if (s->kind == SPH_H_GRID)
    return fail(SPH_ERR_UNSUPPORTED, "set-up from the problem statement takes an analytic "
                                     "sizing; give gridded sizing's particles to "
                                     "sph_mesh_create_with_particles");
  if (p->init != SPH_INIT_DENSITY && p->init != SPH_INIT_UNIFORM)
    return fail(SPH_ERR_INVALID_ARG, "init must be SPH_INIT_DENSITY or SPH_INIT_UNIFORM");
  if (p->n_particles < 0 || p->n_particles > 0x7ffffff0ll)
    return fail(SPH_ERR_INVALID_ARG, "n_particles out of range");
  const int D = g->dim;
  const int res = p->mass_res > 0 ? p->mass_res : (D == 2 ? 1024 : 128);
  if (res > (D == 2 ? 16384 : 1024)) return fail(SPH_ERR_INVALID_ARG, "mass_res too large");
  HostJob J0;
  fill_job(J0, g, s, p, 0, 0);
  const std::vector<double> M = setup::masses(J0.dev.g, J0.feats, res);
  P = setup::plan(J0.feats, M, p->n_particles);
  int64_t total = 0;
  for (size_t f = 0; f < P.count.size(); ++f) {
    if (P.count[f] < 0)
      return fail(SPH_ERR_INVALID_ARG, "feature %zu gets a negative particle count", f);
    total += P.count[f];
  }
  if (total > 0x7ffffff0ll) return fail(SPH_ERR_INVALID_ARG, "too many particles");
  s2 = *s;   // h scaled by P.scale
  s2.h0 = s->h0 * P.scale;
  if (s->kind == SPH_H_LINEAR_FROM_POINT || s->kind == SPH_H_SHELL) s2.grad = s->grad * P.scale;
  if (!want_particles) return SPH_OK;
  HostJob J1;
  fill_job(J1, g, &s2, p, 0, 0);
  double hmin = 0.0, hmax = 0.0, lip = 0.0;
  sizing_bounds(g, &s2, hmin, hmax, lip);
  return setup::sample(J1.dev.g, J1.feats, P, p->init, lip, p->seed, xyz, feat);
}

extern "C" sph_status sph_job_setup(const sph_geometry *g, const sph_sizing *s,
                                    const sph_params *p, double *h_scale, double *h0_scaled,
                                    double *grad_scaled, int64_t *counts, int32_t counts_cap,
                                    int32_t *n_features, double *xyz, int32_t *feature,
                                    int64_t capacity, int64_t *n_out) {
  setup::Plan P;
  sph_sizing s2{};
  std::vector<double> x;
  std::vector<int32_t> f;
  if (sph_status st = problem_setup(g, s, p, xyz != nullptr || feature != nullptr, P, s2, x, f))
    return st;
  const int32_t nf = (int32_t)P.count.size();
  int64_t total = 0;
  for (int64_t c : P.count) total += c;
  if (h_scale) *h_scale = P.scale;
  if (h0_scaled) *h0_scaled = s2.h0;
  if (grad_scaled) *grad_scaled = s2.grad;
  if (n_features) *n_features = nf;
  if (n_out) *n_out = total;
  if (counts) {
    if (counts_cap < nf) return fail(SPH_ERR_INVALID_ARG, "capacity %d < %d features", counts_cap, nf);
    for (int32_t q = 0; q < nf; ++q) counts[q] = P.count[q];
  }
  if (xyz || feature) {
    if (capacity < (int64_t)f.size())
      return fail(SPH_ERR_INVALID_ARG, "capacity %lld < %zu particles", (long long)capacity, f.size());
    if (xyz) std::memcpy(xyz, x.data(), sizeof(double) * x.size());
    if (feature) std::memcpy(feature, f.data(), sizeof(int32_t) * f.size());
  }
  return SPH_OK;
}

// the tag system of a level-set domain's background grid (sec. 3.2)
extern "C" sph_status sph_tags(const sph_geometry *g, int32_t *ctype, int32_t *cindex,
                               int32_t *n_volumes, int32_t *n_patches, int32_t *curve_patches) {
  if (!g) return fail(SPH_ERR_INVALID_ARG, "null geometry");
  // the patches are what this finds: a 3D geometry may leave them unset
  sph_geometry gg = *g;
  std::vector<int32_t> unset;
  if (gg.dim == 3 && gg.n_curves > 0 && (gg.n_patches < 1 || !gg.curve_patches)) {
    unset.assign(2 * (size_t)gg.n_curves, -1);
    gg.n_patches = 1;
    gg.curve_patches = unset.data();
  }
  if (sph_status st = validate_geometry(&gg)) return st;
  if (gg.domain != SPH_DOMAIN_LEVEL_SET)
    return fail(SPH_ERR_INVALID_ARG, "the tag system needs a level-set domain");
  if (!ctype || !cindex || !n_volumes || !n_patches || (gg.n_curves > 0 && !curve_patches))
    return fail(SPH_ERR_INVALID_ARG, "NULL output");
  tags::build(gg.dim, gg.phi_n, gg.phi_lo, gg.phi_hi, gg.phi, gg.n_curves, gg.curve_off,
              gg.curve_pts, gg.n_corners, gg.corners, ctype, cindex, n_volumes, n_patches,
              curve_patches);
  return SPH_OK;
}

extern "C" sph_status sph_mesh_create(const sph_geometry *g, const sph_sizing *s,
                                      const sph_params *p, sph_mesh **out) {
  if (!out) return fail(SPH_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  setup::Plan P;
  sph_sizing s2{};
  std::vector<double> xyz;
  std::vector<int32_t> feat;
  if (sph_status st = problem_setup(g, s, p, true, P, s2, xyz, feat)) return st;
  sph_mesh *m = nullptr;
  if (sph_status st = sph_mesh_create_with_particles(g, &s2, p, (int64_t)feat.size(), xyz.data(),
                                                     feat.data(), &m))
    return st;
  m->h_scale = P.scale;
  m->counts = P.count;
  *out = m;
  return SPH_OK;
}

extern "C" sph_status sph_mesh_setup_info(sph_mesh *m, double *h_scale, int64_t *counts,
                                          int32_t cap, int32_t *n_features) {
  if (!m) return fail(SPH_ERR_INVALID_ARG, "null handle");
  if (h_scale) *h_scale = m->h_scale;
  const int32_t nf = (int32_t)m->counts.size();
  if (n_features) *n_features = nf;
  if (counts) {
    if (cap < nf) return fail(SPH_ERR_INVALID_ARG, "capacity %d < %d features", cap, nf);
    for (int32_t f = 0; f < nf; ++f) counts[f] = m->counts[f];
  }
  return SPH_OK;
}

extern "C" void sph_mesh_destroy(sph_mesh *m) { delete m; }

extern "C" const char *sph_mesh_last_error(void) { return g_err.c_str(); }

extern "C" sph_status sph_mesh_step(sph_mesh *m, int32_t n_steps) {
  if (!m || n_steps < 0) return fail(SPH_ERR_INVALID_ARG, "bad handle or step count");
  return m->b->step(n_steps);
}

extern "C" sph_status sph_mesh_sync(sph_mesh *m) {
  if (!m) return fail(SPH_ERR_INVALID_ARG, "null handle");
  HIPCHK(hipStreamSynchronize(m->b->stream));
  return SPH_OK;
}

extern "C" sph_status sph_mesh_positions(sph_mesh *m, double *xyz, int32_t *feature,
                                         int64_t capacity, int64_t *n_out) {
  if (!m) return fail(SPH_ERR_INVALID_ARG, "null handle");
  return sph_batch_positions(m->b, m->job, xyz, feature, capacity, n_out);
}

extern "C" sph_status sph_mesh_error(sph_mesh *m, double *e_sys, int32_t *phase, int32_t *converged,
                                     int64_t *step) {
  if (!m) return fail(SPH_ERR_INVALID_ARG, "null handle");
  return sph_batch_error(m->b, m->job, e_sys, phase, converged, step);
}

extern "C" sph_status sph_mesh_counters(sph_mesh *m, double *out) {
  if (!m) return fail(SPH_ERR_INVALID_ARG, "null handle");
  return sph_batch_counters(m->b, m->job, out);
}

extern "C" sph_status sph_batch_list_builds(sph_batch *b, int64_t *builds) {
  if (!b || !builds) return fail(SPH_ERR_INVALID_ARG, "null argument");
  unsigned long long v = 0;
  if (b->skin > 0.0) {
    HIPCHK(hipMemcpyAsync(&v, b->vstate + VS_BUILDS, sizeof v, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
  }
  *builds = (int64_t)v;
  return SPH_OK;
}

extern "C" sph_status sph_mesh_list_builds(sph_mesh *m, int64_t *builds) {
  if (!m) return fail(SPH_ERR_INVALID_ARG, "null handle");
  return sph_batch_list_builds(m->b, builds);
}

extern "C" sph_status sph_mesh_velocities(sph_mesh *m, double *vel) {
  if (!m || !vel) return fail(SPH_ERR_INVALID_ARG, "null argument");
  sph_batch *b = m->b;
  HIPCHK(hipStreamSynchronize(b->stream));
  const Parts &s = b->P[b->cur];
  std::vector<uint32_t> oid;
  HIPCHK(pull(oid, s.oid, b->n, b->stream));
  std::vector<double4> v;
  HIPCHK(pull(v, s.v, b->n, b->stream));
  for (int i = 0; i < b->n; ++i) {
    double *o = vel + 3 * (size_t)oid[i];
    o[0] = v[i].x;
    o[1] = v[i].y;
    o[2] = b->D == 3 ? v[i].z : 0.0;
  }
  return SPH_OK;
}

extern "C" sph_status sph_mesh_set_state(sph_mesh *m, const double *xyz, const double *vel) {
  if (!m) return fail(SPH_ERR_INVALID_ARG, "null handle");
  sph_batch *b = m->b;
  HIPCHK(hipStreamSynchronize(b->stream));
  if (b->n == 0) return SPH_OK;
  const Parts &s = b->P[b->cur];
  std::vector<uint32_t> oid;
  HIPCHK(pull(oid, s.oid, b->n, b->stream));
  if (xyz) {
    std::vector<double4> xh(b->n);
    for (int i = 0; i < b->n; ++i) {
      const double *p = xyz + 3 * (size_t)oid[i];
      xh[i] = make_double4(p[0], p[1], b->D == 3 ? p[2] : 0.0, 0.0);
    }
    HIPCHK(hipMemcpyAsync(s.xh, xh.data(), xh.size() * sizeof(double4), hipMemcpyHostToDevice,
                          b->stream));
    // new positions: new h, cells and ranks
    HIPCHK(hipMemsetAsync(b->cnt, 0, sizeof(uint32_t) * b->ncell, b->stream));
    if (sph_status st = b->hash_range(0, b->n)) return st;
    HIPCHK(hipStreamSynchronize(b->stream));
  }
  if (vel) {
    std::vector<double4> v(b->n);
    for (int i = 0; i < b->n; ++i) {
      const double *p = vel + 3 * (size_t)oid[i];
      v[i] = make_double4(p[0], p[1], b->D == 3 ? p[2] : 0.0, 0.0);
    }
    HIPCHK(hipMemcpyAsync(s.v, v.data(), v.size() * sizeof(double4), hipMemcpyHostToDevice,
                          b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
  }
  return SPH_OK;
}

// Lists of every particle at the current positions: sort into cell order,
// build the lists, then re-hash so that the next step starts from consistent
// cell counts.
static sph_status build_lists_now(sph_mesh *m) {
  sph_batch *b = m->b;
  b->invalidate_graph();
  sph_status st = b->force_rebuild();   // a real sort, whatever the Verlet lists' state
  if (!st) st = b->enqueue_sort();
  // with Verlet lists the sorted particles are in the other buffer (a step's
  // list build would copy them back); make it the current one
  if (b->skin > 0.0) b->cur = 1 - b->cur;
  if (!st) st = b->D == 2 ? b->enqueue_lists_only<2>() : b->enqueue_lists_only<3>();
  if (!st) st = b->hash_range(0, b->n);
  if (st) return st;
  HIPCHK(hipStreamSynchronize(b->stream));
  return b->check_job(m->job);
}

extern "C" sph_status sph_mesh_neighbors(sph_mesh *m, int64_t *offsets, int32_t *ids, int8_t *rel,
                                         int64_t cap, int64_t *n_pairs) {
  if (!m || !offsets) return fail(SPH_ERR_INVALID_ARG, "null argument");
  sph_batch *b = m->b;
  HIPCHK(hipStreamSynchronize(b->stream));
  const int n = b->n;
  if (n == 0) {
    offsets[0] = 0;
    if (n_pairs) *n_pairs = 0;
    return SPH_OK;
  }
  sph_status st = build_lists_now(m);
  if (st) return st;
  const Parts &s = b->P[b->cur];
  std::vector<uint32_t> oid, nnb, nbr;
  HIPCHK(pull(oid, s.oid, n, b->stream));
  HIPCHK(pull(nnb, b->nnb, n, b->stream));
  HIPCHK(pull(nbr, b->nbr, (size_t)n * b->cap, b->stream));
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
      uint32_t u = nbr[((size_t)(e / LB) * n + i) * LB + e % LB];
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

extern "C" sph_status sph_mesh_neighbors_of(sph_mesh *m, int32_t count, const int64_t *idx,
                                            int64_t *offsets, int32_t *ids, int8_t *rel,
                                            int64_t cap, int64_t *n_pairs) {
  if (!m || !offsets || (count > 0 && !idx)) return fail(SPH_ERR_INVALID_ARG, "null argument");
  if (count < 0) return fail(SPH_ERR_INVALID_ARG, "count < 0");
  sph_batch *b = m->b;
  HIPCHK(hipStreamSynchronize(b->stream));
  const int n = b->n;
  for (int32_t q = 0; q < count; ++q)
    if (idx[q] < 0 || idx[q] >= n)
      return fail(SPH_ERR_INVALID_ARG, "particle index %lld out of range", (long long)idx[q]);
  offsets[0] = 0;
  if (count == 0) {
    if (n_pairs) *n_pairs = 0;
    return SPH_OK;
  }
  sph_status st = build_lists_now(m);
  if (st) return st;
  const Parts &s = b->P[b->cur];
  std::vector<uint32_t> oid, nnb;
  HIPCHK(pull(oid, s.oid, n, b->stream));
  HIPCHK(pull(nnb, b->nnb, n, b->stream));
  std::vector<int> slot(n);                 // caller id -> cell-order position
  for (int i = 0; i < n; ++i) slot[oid[i]] = i;
  int64_t total = 0;
  for (int32_t q = 0; q < count; ++q) {
    total += nnb[slot[idx[q]]];
    offsets[q + 1] = total;
  }
  if (n_pairs) *n_pairs = total;
  if (!ids && !rel) return SPH_OK;
  if (cap < total) return fail(SPH_ERR_INVALID_ARG, "capacity %lld < %lld pairs", (long long)cap,
                               (long long)total);
  std::vector<uint32_t> row;
  std::vector<std::pair<uint32_t, int8_t>> tmp;
  for (int32_t q = 0; q < count; ++q) {
    const int i = slot[idx[q]];
    const uint32_t k = nnb[i];
    row.assign(((k + LB - 1) / LB) * LB, 0u);
    for (uint32_t blk = 0; blk * LB < k; ++blk)    // one block of LB entries per copy
      HIPCHK(hipMemcpyAsync(row.data() + (size_t)blk * LB, b->nbr + ((size_t)blk * n + i) * LB,
                            sizeof(uint32_t) * LB, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    tmp.clear();
    for (uint32_t e = 0; e < k; ++e)
      tmp.push_back({oid[row[e] & 0x7fffffffu], (int8_t)((row[e] >> 31) ? 2 : 1)});
    std::sort(tmp.begin(), tmp.end());
    for (size_t t = 0; t < tmp.size(); ++t) {
      if (ids) ids[offsets[q] + t] = (int32_t)tmp[t].first;
      if (rel) rel[offsets[q] + t] = tmp[t].second;
    }
  }
  return SPH_OK;
}

extern "C" sph_status sph_mesh_field(sph_mesh *m, int32_t which, double *out) {
  if (!m || !out) return fail(SPH_ERR_INVALID_ARG, "null argument");
  sph_batch *b = m->b;
  if (which < 0 || which > 5) return fail(SPH_ERR_INVALID_ARG, "unknown field %d", which);
  if (which >= 3 && !b->debug) return fail(SPH_ERR_INVALID_ARG, "field %d needs debug_fields", which);
  HIPCHK(hipStreamSynchronize(b->stream));
  const int n = b->n;
  const Parts &s = b->P[b->cur];
  std::vector<uint32_t> oid;
  HIPCHK(pull(oid, s.oid, n, b->stream));
  std::vector<double> col;
  auto scatter1 = [&]() {
    for (int i = 0; i < n; ++i) out[oid[i]] = col[i];
  };
  auto scatter4 = [&](const std::vector<double4> &v) {
    for (int i = 0; i < n; ++i) {
      double *o = out + 3 * (size_t)oid[i];
      o[0] = v[i].x;
      o[1] = v[i].y;
      o[2] = b->D == 3 ? v[i].z : 0.0;
    }
  };
  std::vector<double4> v4;
  switch (which) {
    case 0: {
      HIPCHK(pull(v4, s.xh, n, b->stream));
      col.resize(n);
      for (int i = 0; i < n; ++i) col[i] = v4[i].w;
      scatter1();
      break;
    }
    case 3: HIPCHK(pull(col, b->dbg_vt, n, b->stream)); scatter1(); break;
    case 4: HIPCHK(pull(col, b->dbg_gam, n, b->stream)); scatter1(); break;
    case 5: HIPCHK(pull(v4, b->dbg_vm, n, b->stream)); scatter4(v4); break;
    default: {
      const void *src = which == 1 ? b->ap : b->acc;
      if (b->prec == SPH_FP64) {
        HIPCHK(pull(v4, src, n, b->stream));
      } else {
        std::vector<float4> f4;
        HIPCHK(pull(f4, src, n, b->stream));
        v4.resize(n);
        for (int i = 0; i < n; ++i) v4[i] = make_double4(f4[i].x, f4[i].y, f4[i].z, f4[i].w);
      }
      scatter4(v4);
    }
  }
  return SPH_OK;
}

extern "C" sph_status sph_mesh_group_state(sph_mesh *m, int32_t f, double *out) {
  if (!m || !out || f < 0 || f >= MAXF) return fail(SPH_ERR_INVALID_ARG, "bad argument");
  sph_batch *b = m->b;
  HIPCHK(hipStreamSynchronize(b->stream));
  Group G;
  HIPCHK(hipMemcpyAsync(&G, b->d_grp + m->job * MAXF + f, sizeof G, hipMemcpyDeviceToHost, b->stream));
  HIPCHK(hipStreamSynchronize(b->stream));
  out[0] = G.phase; out[1] = G.n_ph; out[2] = G.esys; out[3] = G.dt1; out[4] = G.dt;
  out[5] = G.vbar; out[6] = G.reset_next; out[7] = G.a_last; out[8] = G.a_prev; out[9] = G.nwin;
  return SPH_OK;
}

extern "C" int64_t sph_mesh_device_bytes(sph_mesh *m) { return m ? (int64_t)m->b->bytes : 0; }

extern "C" sph_status sph_mesh_profile(sph_mesh *m, int32_t enable) {
  if (!m) return fail(SPH_ERR_INVALID_ARG, "null handle");
  sph_batch *b = m->b;
  HIPCHK(hipStreamSynchronize(b->stream));
  for (auto &e : b->ev_live) {
    b->ev_pool.push_back(e.a);
    b->ev_pool.push_back(e.b);
  }
  b->ev_live.clear();
  for (int k = 0; k < KID_COUNT; ++k) {
    b->kms[k] = 0.0;
    b->kcount[k] = 0;
  }
  b->profiling = enable != 0;
  return SPH_OK;
}

extern "C" sph_status sph_mesh_kernel_stats(sph_mesh *m, int32_t kid, double *ms, int64_t *launches) {
  if (!m || kid < 0 || kid >= KID_COUNT) return fail(SPH_ERR_INVALID_ARG, "bad argument");
  sph_batch *b = m->b;
  HIPCHK(hipStreamSynchronize(b->stream));
  for (auto &e : b->ev_live) {
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, e.a, e.b));
    b->kms[e.kid] += t;
    b->kcount[e.kid] += 1;
    b->ev_pool.push_back(e.a);
    b->ev_pool.push_back(e.b);
  }
  b->ev_live.clear();
  if (ms) *ms = b->kms[kid];
  if (launches) *launches = b->kcount[kid];
  return SPH_OK;
}

extern "C" int32_t sph_mesh_kernel_count(void) { return KID_COUNT; }

extern "C" const char *sph_mesh_kernel_name(int32_t kid) {
  return kid >= 0 && kid < KID_COUNT ? kKernelNames[kid] : "";
}

// the longest series a control replay takes
constexpr int32_t kReplayMax = 1000000;

// arguments of a control replay checked, and the control record built
static sph_status replay_setup(const sph_params *p, int32_t n, bool bufs, Ctl &C) {
  if (n > kReplayMax)
    return fail(SPH_ERR_INVALID_ARG, "series of %d steps exceeds the maximum of %d", n, kReplayMax);
  if (!p || n < 0 || (n && !bufs)) return fail(SPH_ERR_INVALID_ARG, "bad argument");
  if (p->window_samples < 1 || p->window_samples > MAXRING || p->sample_every < 1 ||
      p->reset_period < 1 || p->ramp_halving < 1 || p->ramp_steps < 1)
    return fail(SPH_ERR_INVALID_ARG, "bad control parameters");
  C = Ctl{};
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
  return SPH_OK;
}

extern "C" sph_status sph_mesh_control_replay(const sph_params *p, int32_t n, const double *vbar,
                                              const double *dt, int32_t *phase, int32_t *reset,
                                              double *e_sys) {
  Ctl C;
  if (sph_status st = replay_setup(p, n, vbar && dt && phase && reset && e_sys, C)) return st;
  void *buf = nullptr;
  const size_t nn = std::max(n, 1);
  const size_t bytes = sizeof(Group) + nn * (8 + 8 + 4 + 4 + 8);
  HIPCHK(hipMalloc(&buf, bytes));
  char *b = (char *)buf;
  Group *dg = (Group *)b;     // the control state (the kernel initialises it)
  double *dv = (double *)(b + sizeof(Group));
  double *dd = dv + nn;
  double *de = dd + nn;
  int32_t *dp = (int32_t *)(de + nn);
  int32_t *dr = dp + nn;
  hipError_t e = hipSuccess;
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

// ---------------------------------------------------------------------------
// Control replay without allocation.  Its only scratch is the control state
// the replay kernel evolves (one Group); it lives in this file-scope device
// array, one copy per GPU for the life of the process.  In host code the
// array's name is not a device address: each device's address is looked up
// once with hipGetSymbolAddress (with that device current) and kept.
static __device__ __align__(256) Group scratch[1];
static_assert(sizeof(Group) <= 768, "the no-allocation scratch is documented as ~700 bytes");

static std::mutex g_scratch_mu;
static Group *g_scratch_dev[64];   // address of scratch on device d, or null

static sph_status scratch_on_current_device(Group **out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(SPH_ERR_UNSUPPORTED, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(SPH_ERR_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_dev[dev] = static_cast<Group *>(ptr);
  }
  *out = g_scratch_dev[dev];
  return SPH_OK;
}

extern "C" sph_status sph_mesh_control_replay_noalloc(const sph_params *p, int32_t n,
                                                      const double *vbar, const double *dt,
                                                      int32_t *phase, int32_t *reset,
                                                      double *e_sys, void *stream) {
  Ctl C;
  if (sph_status st = replay_setup(p, n, vbar && dt && phase && reset && e_sys, C)) return st;
  Group *state = nullptr;
  if (sph_status st = scratch_on_current_device(&state)) return st;
  hipLaunchKernelGGL(k_control_replay, dim3(1), dim3(64), 0, (hipStream_t)stream, C, n, vbar, dt,
                     phase, reset, e_sys, state);
  HIPCHK(hipGetLastError());
  return SPH_OK;
}
