// sph_setup.h -- Algorithm 1's set-up from the problem statement, on the
// host: the target information of every feature (sec. 3.2: its mass, the
// integral of the target density rho_t = h^-k over the feature, k its
// intrinsic dimension), the particle budget split over the features by those
// masses at unit particle mass, and the initial particles, drawn with
// probability proportional to rho_t from a Mersenne Twister (sec. 3.6).
//
// The budget n_particles rarely equals the sum of the masses at the given
// h_t, so h is scaled by the factor s that makes sum_k M_k / s^k equal the
// budget (reading R25); s is found by bisection in log s.  n_particles = 0
// keeps h_t and takes the rounded masses as the counts.
//
// Masses are midpoint sums: the volume on a res^D grid over the box (points
// inside the domain), the box sides on res^(D-1) grids (4 res points per
// side in 2D), circles on 4 res points, spheres on res x 2 res equal-area
// bands, ellipses and ellipsoids on the same points of the unit circle or
// sphere mapped by the semi-axes with their measure factor, 3D box edges on
// 4 res points.  Counts are round(M_k / s^k) (half to even), the volume
// taking the remainder; every box corner holds one fixed particle.
#pragma once
#include <random>

namespace sph {
namespace setup {

enum { INIT_DENSITY = 0, INIT_UNIFORM = 1 };

// uniform doubles in [0, 1) from the 64-bit Mersenne Twister (53 random bits)
struct Rng {
  std::mt19937_64 g;
  explicit Rng(uint64_t seed) : g(seed) {}
  double u() { return (double)(g() >> 11) * 0x1.0p-53; }
  double normal() {   // Marsaglia's polar method
    for (;;) {
      const double a = 2.0 * u() - 1.0, b = 2.0 * u() - 1.0, s = a * a + b * b;
      if (s > 0.0 && s < 1.0) return a * std::sqrt(-2.0 * std::log(s) / s);
    }
  }
};

inline double h_at(const Geom &G, const double *p) {
  return G.dim == 2 ? h_target<2>(G, p) : h_target<3>(G, p);
}
inline bool in_domain(const Geom &G, const double *p) {
  return G.dim == 2 ? inside<2>(G, p) : inside<3>(G, p);
}

// unit vectors of the midpoint rule on the circle (4 res points) or of res x
// 2 res equal-area bands on the sphere, each with its share of the full
// angle (2 pi or 4 pi)
inline void sphere_rule(int D, int res, std::vector<double> &u, double &dOmega) {
  u.clear();
  if (D == 2) {
    const int nseg = 4 * res;
    for (int q = 0; q < nseg; ++q) {
      const double th = (q + 0.5) * 2.0 * M_PI / nseg;
      u.insert(u.end(), {std::cos(th), std::sin(th), 0.0});
    }
    dOmega = 2.0 * M_PI / nseg;
    return;
  }
  for (int i = 0; i < res; ++i) {
    const double ct = -1.0 + (i + 0.5) * 2.0 / res;
    const double st = std::sqrt(1.0 - ct * ct);
    for (int j = 0; j < 2 * res; ++j) {
      const double ph = (j + 0.5) * M_PI / res;
      u.insert(u.end(), {st * std::cos(ph), st * std::sin(ph), ct});
    }
  }
  dOmega = 4.0 * M_PI / (2.0 * res * res);
}

// point of hole q's boundary for the unit vector u (c + R^T (a u)) and the
// boundary measure per unit solid angle there (prod(a) |u / a|)
inline void hole_point(const Geom &G, int q, const double *u, double *p, double &meas) {
  const int D = G.dim;
  double au[3] = {0.0, 0.0, 0.0}, prod = 1.0, s = 0.0;
  for (int k = 0; k < D; ++k) {
    const double a = G.ha[q][k];
    au[k] = a * u[k];
    prod *= a;
    s += (u[k] / a) * (u[k] / a);
  }
  for (int m = 0; m < 3; ++m) {
    double v = 0.0;
    if (m < D)
      for (int k = 0; k < D; ++k) v += G.hR[q][3 * k + m] * au[k];
    p[m] = m < D ? G.hc[q][m] + v : 0.0;
  }
  meas = prod * std::sqrt(s);
}

struct Plan {
  std::vector<double> mass;     // per feature, at the unscaled h_t
  std::vector<int64_t> count;   // particles per feature
  double scale = 1.0;           // s: h is multiplied by it
};

// masses of every feature at the sizing of G (the same quadrature points for
// every sizing)
inline std::vector<double> masses(const Geom &G, const std::vector<HFeat> &F, int res) {
  const int D = G.dim;
  std::vector<double> M(F.size(), 0.0);
  const int nseg = 4 * res;
  double p[3] = {0.0, 0.0, 0.0};
  std::vector<double> u;
  double dOmega = 0.0;
  for (size_t f = 0; f < F.size(); ++f) {
    const HFeat &H = F[f];
    double sum = 0.0;
    if (H.kind == K_VOL) {
      double cellv = 1.0;
      for (int a = 0; a < D; ++a) cellv *= (G.hi[a] - G.lo[a]) / res;
      const int nz = D == 3 ? res : 1;
      for (int k = 0; k < nz; ++k)
        for (int j = 0; j < res; ++j)
          for (int i = 0; i < res; ++i) {
            const int id[3] = {i, j, k};
            for (int a = 0; a < 3; ++a)
              p[a] = a < D ? G.lo[a] + (id[a] + 0.5) * (G.hi[a] - G.lo[a]) / res : 0.0;
            if (!in_domain(G, p)) continue;
            sum += std::pow(h_at(G, p), -(double)D);
          }
      M[f] = sum * cellv;
    } else if (H.kind == K_BOXSIDE) {
      const int a = H.axis;
      if (D == 2) {
        const int o = 1 - a;
        p[a] = H.side ? G.hi[a] : G.lo[a];
        p[2] = 0.0;
        for (int q = 0; q < nseg; ++q) {
          p[o] = G.lo[o] + (q + 0.5) * (G.hi[o] - G.lo[o]) / nseg;
          sum += 1.0 / h_at(G, p);
        }
        M[f] = sum * (G.hi[o] - G.lo[o]) / nseg;
      } else {
        const int o1 = a == 0 ? 1 : 0, o2 = a == 2 ? 1 : 2;
        p[a] = H.side ? G.hi[a] : G.lo[a];
        for (int i = 0; i < res; ++i)
          for (int j = 0; j < res; ++j) {
            p[o1] = G.lo[o1] + (i + 0.5) * (G.hi[o1] - G.lo[o1]) / res;
            p[o2] = G.lo[o2] + (j + 0.5) * (G.hi[o2] - G.lo[o2]) / res;
            const double h = h_at(G, p);
            sum += 1.0 / (h * h);
          }
        M[f] = sum * (G.hi[o1] - G.lo[o1]) * (G.hi[o2] - G.lo[o2]) / ((double)res * res);
      }
    } else if (H.kind == K_HOLE || H.kind == K_SHELL) {
      sphere_rule(D, res, u, dOmega);
      const size_t np = u.size() / 3;
      for (size_t t = 0; t < np; ++t) {
        double meas;
        if (H.kind == K_SHELL) {
          for (int a = 0; a < 3; ++a) p[a] = a < D ? G.dc[a] + G.dR * u[3 * t + a] : 0.0;
          meas = D == 2 ? G.dR : G.dR * G.dR;
        } else {
          hole_point(G, H.hole, &u[3 * t], p, meas);
        }
        sum += std::pow(h_at(G, p), -(double)(D - 1)) * meas * dOmega;
      }
      M[f] = sum;
    } else if (H.kind == K_EDGE3) {
      const int a = H.axis;
      p[H.fax[0]] = H.fsd[0] ? G.hi[H.fax[0]] : G.lo[H.fax[0]];
      p[H.fax[1]] = H.fsd[1] ? G.hi[H.fax[1]] : G.lo[H.fax[1]];
      for (int q = 0; q < nseg; ++q) {
        p[a] = G.lo[a] + (q + 0.5) * (G.hi[a] - G.lo[a]) / nseg;
        sum += 1.0 / h_at(G, p);
      }
      M[f] = sum * (G.hi[a] - G.lo[a]) / nseg;
    }
  }
  return M;
}

// the particle counts of every feature for the budget n_total (0: the masses
// as they are)
inline Plan plan(const std::vector<HFeat> &F, const std::vector<double> &M, int64_t n_total) {
  Plan P;
  P.mass = M;
  int64_t ncorner = 0;
  for (const HFeat &H : F) ncorner += H.type == T_SI ? 1 : 0;
  auto total = [&](double s) {
    double t = (double)ncorner;
    for (size_t f = 0; f < F.size(); ++f)
      if (F[f].type != T_SI) t += M[f] / std::pow(s, (double)F[f].k);
    return t;
  };
  if (n_total > 0) {
    double lo = 1e-3, hi = 1e3;
    for (int it = 0; it < 200; ++it) {
      const double mid = std::sqrt(lo * hi);
      if (total(mid) > (double)n_total) lo = mid; else hi = mid;
    }
    P.scale = std::sqrt(lo * hi);
  }
  P.count.assign(F.size(), 0);
  int64_t placed = 0;
  for (size_t f = 0; f < F.size(); ++f) {
    if (F[f].type == T_SI) {
      P.count[f] = 1;
      continue;
    }
    P.count[f] = (int64_t)std::nearbyint(M[f] / std::pow(P.scale, (double)F[f].k));
    placed += P.count[f];
  }
  if (n_total > 0) P.count[0] += n_total - ncorner - placed;
  return P;
}

// Initial particles of every feature: proposals uniform on the feature (for
// the volume: a cell of an envelope grid chosen by weight, then a point
// uniform in it), kept with probability (h_lb / h)^k, so that the kept points
// have density proportional to rho_t = h^-k (INIT_DENSITY); INIT_UNIFORM
// keeps every proposal inside the domain.  h_lb is h0 on the lower-
// dimensional features and, for the volume, a lower bound of h over the
// cell from the Lipschitz constant L of h_t: max(h0, h(centre) - L r), r the
// cell's half-diagonal.  Cells that lie wholly outside the domain (inside a
// hole, or outside the ball domain) get no weight.
inline sph_status sample(const Geom &G, const std::vector<HFeat> &F, const Plan &P, int init,
                         double lip, uint64_t seed, std::vector<double> &xyz,
                         std::vector<int32_t> &feat) {
  const int D = G.dim;
  Rng rng(seed);
  const double h0 = G.h0;
  xyz.clear();
  feat.clear();
  auto keep = [&](double h, int k) {
    if (init == INIT_UNIFORM) return true;
    return rng.u() < std::pow(h0 / h, (double)k);
  };
  auto push = [&](const double *p, int f) {
    xyz.insert(xyz.end(), {p[0], p[1], D == 3 ? p[2] : 0.0});
    feat.push_back(f);
  };
  // a proposal budget far above any sane acceptance; exceeding it is an error
  auto budget = [&](int64_t want) { return std::max<int64_t>(1 << 20, 100000 * want); };
  for (size_t f = 0; f < F.size(); ++f) {
    const HFeat &H = F[f];
    const int64_t want = P.count[f];
    double p[3] = {0.0, 0.0, 0.0};
    if (H.kind == K_VOL) {
      const int g = D == 2 ? 128 : 48;
      double side[3] = {0.0, 0.0, 0.0}, r2 = 0.0;
      for (int a = 0; a < D; ++a) {
        side[a] = (G.hi[a] - G.lo[a]) / g;
        r2 += 0.25 * side[a] * side[a];
      }
      const double r = std::sqrt(r2);
      const int ncell = D == 2 ? g * g : g * g * g;
      std::vector<double> cum(ncell), hlb(ncell);
      double acc = 0.0;
      for (int c = 0; c < ncell; ++c) {
        const int id[3] = {c % g, (c / g) % g, c / (g * g)};
        double cen[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < D; ++a) cen[a] = G.lo[a] + (id[a] + 0.5) * side[a];
        double w = 1.0;
        bool out = false;
        if (G.domain == SPH_DOMAIN_BALL) {
          double s = 0.0;
          for (int a = 0; a < D; ++a) s += (cen[a] - G.dc[a]) * (cen[a] - G.dc[a]);
          out = std::sqrt(s) - r >= G.dR;
        } else {
          for (int q = 0; q < G.nh && !out; ++q) {
            double y[3] = {0.0, 0.0, 0.0};
            if (D == 2) ell_local<2>(G, q, cen, y); else ell_local<3>(G, q, cen, y);
            const double lev = D == 2 ? ell_level<2>(G, q, y) : ell_level<3>(G, q, y);
            out = std::sqrt(lev) + r / G.hamin[q] <= 1.0 - 1e-9;
          }
        }
        const double hl = std::max(h0, h_at(G, cen) - lip * r);
        hlb[c] = hl;
        if (out) w = 0.0;
        else if (init != INIT_UNIFORM) w = std::pow(hl, -(double)D);
        acc += w;
        cum[c] = acc;
      }
      if (!(acc > 0.0)) return fail(SPH_ERR_INVALID_ARG, "the domain has no volume");
      int64_t got = 0, tries = 0;
      while (got < want) {
        if (++tries > budget(want)) return fail(SPH_ERR_INVALID_ARG, "volume sampling did not converge");
        const double t = rng.u() * acc;
        const int c = (int)(std::upper_bound(cum.begin(), cum.end(), t) - cum.begin());
        if (c >= ncell) continue;
        const int id[3] = {c % g, (c / g) % g, c / (g * g)};
        for (int a = 0; a < D; ++a) p[a] = G.lo[a] + (id[a] + rng.u()) * side[a];
        if (!in_domain(G, p)) continue;
        if (init != INIT_UNIFORM && !(rng.u() < std::pow(hlb[c] / h_at(G, p), (double)D))) continue;
        push(p, (int)f);
        ++got;
      }
    } else if (H.type == T_SI) {
      for (int a = 0; a < D; ++a) p[a] = ((H.bits >> a) & 1) ? G.hi[a] : G.lo[a];
      push(p, (int)f);
    } else {
      int64_t got = 0, tries = 0;
      while (got < want) {
        if (++tries > budget(want)) return fail(SPH_ERR_INVALID_ARG, "feature %zu: sampling did not converge", f);
        if (H.kind == K_BOXSIDE || H.kind == K_EDGE3) {
          for (int a = 0; a < D; ++a) p[a] = G.lo[a] + rng.u() * (G.hi[a] - G.lo[a]);
          if (H.kind == K_BOXSIDE) {
            p[H.axis] = H.side ? G.hi[H.axis] : G.lo[H.axis];
          } else {
            p[H.fax[0]] = H.fsd[0] ? G.hi[H.fax[0]] : G.lo[H.fax[0]];
            p[H.fax[1]] = H.fsd[1] ? G.hi[H.fax[1]] : G.lo[H.fax[1]];
          }
        } else {   // a hole's boundary or the ball domain's sphere
          double u[3] = {0.0, 0.0, 0.0}, s = 0.0;
          for (int a = 0; a < D; ++a) {
            u[a] = rng.normal();
            s += u[a] * u[a];
          }
          s = std::sqrt(s);
          for (int a = 0; a < D; ++a) u[a] /= s;
          if (H.kind == K_SHELL) {
            for (int a = 0; a < D; ++a) p[a] = G.dc[a] + G.dR * u[a];
          } else {
            double meas;
            hole_point(G, H.hole, u, p, meas);
            // uniform directions mapped by the semi-axes: thin by the
            // measure factor |u / a| / max |u / a| = min(a) |u / a|
            if (G.hell[H.hole] && !(rng.u() < G.hamin[H.hole] * meas / (G.ha[H.hole][0] * G.ha[H.hole][1] *
                                                                        (D == 3 ? G.ha[H.hole][2] : 1.0))))
              continue;
          }
        }
        if (!keep(h_at(G, p), H.k)) continue;
        push(p, (int)f);
        ++got;
      }
    }
  }
  return SPH_OK;
}

}  // namespace setup
}  // namespace sph
