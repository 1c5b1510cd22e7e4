// The tag system of a level-set domain's background grid (paper sec. 3.2):
// every grid cell gets a type (negative C-, positive C+, surface C_s, curve
// C_c, singular C_si) and the index of its feature within that type, so
// that the zero set's patches, the curves between them and the volumes can
// be told apart.  Host C++; one pass over the cells per step below.
//
//   1. node signs: C+ when phi > 0 at every node of the cell, C- when
//      phi < 0 at every node, C_s otherwise;
//   2. curves, in order: each segment is walked in steps of at most a
//      quarter of the smallest cell side (ceil(length / (side / 4)) steps,
//      both ends included); the cell of every point and its face neighbours
//      become C_c of that curve unless an earlier curve holds them;
//   3. corners, in order: the corner's cell and its 3^D - 1 neighbours
//      become C_si of that corner unless an earlier corner holds them;
//   4. the remaining C_s cells form patches and the C+ cells volumes: the
//      components under face adjacency, numbered in the order of their first
//      cell (x fastest, then y, then z);
//   5. the patches beside curve c: those with a cell that is a face
//      neighbour of one of c's cells.
#pragma once

#include <cmath>
#include <cstdint>
#include <vector>

namespace tags {

enum : int32_t { C_NEG = 0, C_POS = 1, C_SURF = 2, C_CURVE = 3, C_SING = 4 };

struct Grid {
  int D;
  int64_t nc[3];     // cells per axis (1 on the third axis in 2D)
  double lo[3], s[3];
  int64_t cells() const { return nc[0] * nc[1] * nc[2]; }
  int64_t id(int64_t i, int64_t j, int64_t k) const { return (k * nc[1] + j) * nc[0] + i; }
  bool in(int64_t i, int64_t j, int64_t k) const {
    return i >= 0 && j >= 0 && k >= 0 && i < nc[0] && j < nc[1] && k < nc[2];
  }
  // the cell holding x, clamped to the grid
  void cell(const double *x, int64_t *c) const {
    for (int a = 0; a < 3; ++a) {
      c[a] = 0;
      if (a >= D) continue;
      double u = std::floor((x[a] - lo[a]) * s[a]);
      if (!(u > 0.0)) u = 0.0;
      if (u > (double)(nc[a] - 1)) u = (double)(nc[a] - 1);
      c[a] = (int64_t)u;
    }
  }
};

// union-find over cell ids: the smaller id is the root, so that a
// component's root is its first cell
struct Forest {
  std::vector<int64_t> up;
  explicit Forest(int64_t n) : up((size_t)n) {
    for (int64_t v = 0; v < n; ++v) up[(size_t)v] = v;
  }
  int64_t root(int64_t v) {
    while (up[(size_t)v] != v) {
      up[(size_t)v] = up[(size_t)up[(size_t)v]];
      v = up[(size_t)v];
    }
    return v;
  }
  void join(int64_t a, int64_t b) {
    a = root(a);
    b = root(b);
    if (a == b) return;
    if (a < b) up[(size_t)b] = a; else up[(size_t)a] = b;
  }
};

// components of the cells of type t (steps 4); returns their count
inline int32_t components(const Grid &G, const int32_t *type, int32_t *index, int32_t t) {
  Forest F(G.cells());
  for (int64_t k = 0; k < G.nc[2]; ++k)
    for (int64_t j = 0; j < G.nc[1]; ++j)
      for (int64_t i = 0; i < G.nc[0]; ++i) {
        const int64_t v = G.id(i, j, k);
        if (type[v] != t) continue;
        // join with the lower neighbours only: every face pair once
        if (i > 0 && type[v - 1] == t) F.join(v, v - 1);
        if (j > 0 && type[v - G.nc[0]] == t) F.join(v, v - G.nc[0]);
        if (k > 0 && type[v - G.nc[0] * G.nc[1]] == t) F.join(v, v - G.nc[0] * G.nc[1]);
      }
  // roots are first cells, met in increasing order
  std::vector<int32_t> label((size_t)G.cells(), -1);
  int32_t count = 0;
  for (int64_t v = 0; v < G.cells(); ++v) {
    if (type[v] != t) continue;
    const int64_t r = F.root(v);
    if (r == v) label[(size_t)v] = count++;
    index[v] = label[(size_t)r];
  }
  return count;
}

// the tag system of level set phi (nodes n[0] x n[1] x n[2], x fastest, over
// [plo, phi] per axis) with the given curves and corners; type, index: one
// entry per cell; pat: 2 per curve
inline void build(int D, const int32_t *n, const double *plo, const double *phi_hi,
                  const double *phi, int ncurves, const int32_t *coff, const double *cpts,
                  int ncorners, const double *corners, int32_t *type, int32_t *index,
                  int32_t *n_volumes, int32_t *n_patches, int32_t *pat) {
  Grid G{};
  G.D = D;
  for (int a = 0; a < 3; ++a) {
    G.nc[a] = a < D ? (int64_t)n[a] - 1 : 1;
    G.lo[a] = plo[a];
    G.s[a] = a < D ? (double)(n[a] - 1) / (phi_hi[a] - plo[a]) : 0.0;
  }
  const int64_t nx = n[0], nxy = (int64_t)n[0] * n[1];
  // 1. node signs, from the smallest and largest node value
  for (int64_t k = 0; k < G.nc[2]; ++k)
    for (int64_t j = 0; j < G.nc[1]; ++j)
      for (int64_t i = 0; i < G.nc[0]; ++i) {
        double lo_v = INFINITY, hi_v = -INFINITY;
        for (int dk = 0; dk < (D == 3 ? 2 : 1); ++dk)
          for (int dj = 0; dj < 2; ++dj)
            for (int di = 0; di < 2; ++di) {
              const double v = phi[(k + dk) * nxy + (j + dj) * nx + (i + di)];
              lo_v = std::fmin(lo_v, v);
              hi_v = std::fmax(hi_v, v);
            }
        const int64_t v = G.id(i, j, k);
        type[v] = lo_v > 0.0 ? C_POS : (hi_v < 0.0 ? C_NEG : C_SURF);
        index[v] = -1;
      }
  // 2. curves
  double side = INFINITY;
  for (int a = 0; a < D; ++a) side = std::fmin(side, (phi_hi[a] - plo[a]) / (double)G.nc[a]);
  std::vector<char> held((size_t)G.cells(), 0);   // a curve already holds the cell
  for (int c = 0; c < ncurves; ++c)
    for (int32_t e = coff[c]; e + 1 < coff[c + 1]; ++e) {
      const double *p0 = cpts + 3 * (size_t)e, *p1 = p0 + 3;
      double d[3] = {0.0, 0.0, 0.0}, len2 = 0.0;
      for (int a = 0; a < D; ++a) {
        d[a] = p1[a] - p0[a];
        len2 = len2 + d[a] * d[a];
      }
      int64_t steps = (int64_t)std::ceil(std::sqrt(len2) / (0.25 * side));
      if (steps < 1) steps = 1;
      for (int64_t q = 0; q <= steps; ++q) {
        const double f = (double)q / (double)steps;
        double x[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < D; ++a) x[a] = p0[a] + f * d[a];
        int64_t cc[3];
        G.cell(x, cc);
        // the cell itself, then its 2 D face neighbours
        for (int m = 0; m <= 2 * D; ++m) {
          int64_t o[3] = {cc[0], cc[1], cc[2]};
          if (m > 0) o[(m - 1) / 2] += (m & 1) ? -1 : 1;
          if (!G.in(o[0], o[1], o[2])) continue;
          const int64_t v = G.id(o[0], o[1], o[2]);
          if (held[(size_t)v]) continue;
          held[(size_t)v] = 1;
          type[v] = C_CURVE;
          index[v] = c;
        }
      }
    }
  // 3. corners
  std::vector<char> taken((size_t)G.cells(), 0);
  for (int m = 0; m < ncorners; ++m) {
    int64_t cc[3];
    G.cell(corners + 3 * (size_t)m, cc);
    const int64_t r2 = D == 3 ? 1 : 0;
    for (int64_t dk = -r2; dk <= r2; ++dk)
      for (int64_t dj = -1; dj <= 1; ++dj)
        for (int64_t di = -1; di <= 1; ++di) {
          if (!G.in(cc[0] + di, cc[1] + dj, cc[2] + dk)) continue;
          const int64_t v = G.id(cc[0] + di, cc[1] + dj, cc[2] + dk);
          if (taken[(size_t)v]) continue;
          taken[(size_t)v] = 1;
          type[v] = C_SING;
          index[v] = m;
        }
  }
  // 4. patches and volumes
  *n_patches = components(G, type, index, C_SURF);
  *n_volumes = components(G, type, index, C_POS);
  // 5. the patches beside each curve
  std::vector<std::vector<int32_t>> beside((size_t)ncurves);
  for (int64_t k = 0; k < G.nc[2]; ++k)
    for (int64_t j = 0; j < G.nc[1]; ++j)
      for (int64_t i = 0; i < G.nc[0]; ++i) {
        const int64_t v = G.id(i, j, k);
        if (type[v] != C_CURVE) continue;
        std::vector<int32_t> &B = beside[(size_t)index[v]];
        for (int m = 1; m <= 2 * D; ++m) {
          int64_t o[3] = {i, j, k};
          o[(m - 1) / 2] += (m & 1) ? -1 : 1;
          if (!G.in(o[0], o[1], o[2])) continue;
          const int64_t w = G.id(o[0], o[1], o[2]);
          if (type[w] != C_SURF) continue;
          bool have = false;
          for (int32_t p : B) have = have || p == index[w];
          if (!have) B.push_back(index[w]);
        }
      }
  for (int c = 0; c < ncurves; ++c) {
    std::vector<int32_t> &B = beside[(size_t)c];
    if (B.size() > 2) {
      pat[2 * c] = -2;
      pat[2 * c + 1] = -1;
      continue;
    }
    if (B.size() == 2 && B[1] < B[0]) std::swap(B[0], B[1]);
    pat[2 * c] = B.size() > 0 ? B[0] : -1;
    pat[2 * c + 1] = B.size() > 1 ? B[1] : -1;
  }
}

}  // namespace tags
