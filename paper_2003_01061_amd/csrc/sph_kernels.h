// sph_kernels.h -- the gfx950 kernels of one relaxation step.
//
// Per step (Algorithm 1's loop body, every feature at once, all reading x^n):
//   k_hash_count   h_i = h_t(x_i), cell of x_i, rank inside the cell (atomic)
//   k_scan_*       exclusive scan of the cell counts -> cell start table
//   k_scatter      slot of every particle in cell order
//   k_cellsort     order inside a cell by caller id (canonical, history free)
//   k_gather       permute the particle columns into the new order
//   k_neighbors    ELL neighbour list: exact FP64 predicate + feature relation
//   k_sweep_a      Shepard gamma, V~, pressure force with the boundary term,
//                  tangent projection -> a^p; group min of dt_1, sum of V~
//   k_sweep_b      mid-point velocity on the fly, viscous force -> a;
//                  group min of dt
//   k_integrate    v_{n+1/2}, x_{n+1}, projection / rejection, v_{n+1}
//   k_control      E_sys, phases, resets, damping of every feature (1 block)
#pragma once
#include "sph_device.h"

namespace sph {

// ---------------------------------------------------------------------------
// wave-level per-group reductions: lanes of one wave usually share a group;
// each distinct group among the valid lanes is reduced with xor shuffles and
// committed by one lane with a device atomic (min of non-negative double bit
// patterns and integer sums are exact and order independent).
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long umin64(unsigned long long a, unsigned long long b) {
  return a < b ? a : b;
}

// Per-group reduction of one block: every wave reduces each distinct group
// among its valid lanes with xor shuffles, one lane folds the result into the
// block's LDS slot with an LDS atomic, and the block writes one partial per
// group.  Device-wide same-address atomics are avoided on purpose: with
// thousands of waves they serialise.
__device__ __forceinline__ void block_group_reduce(bool valid, int g, unsigned long long vmin,
                                                   unsigned long long vadd,
                                                   unsigned long long *s_min,
                                                   unsigned long long *s_sum, int nf,
                                                   unsigned long long *pmin,
                                                   unsigned long long *psum) {
  for (int t = threadIdx.x; t < nf; t += blockDim.x) {
    s_min[t] = ~0ull;
    s_sum[t] = 0ull;
  }
  __syncthreads();
  unsigned long long mask = __ballot(valid);
  const int lane = __lane_id();
  while (mask) {
    int leader = __ffsll((long long)mask) - 1;
    int gl = __shfl(g, leader);
    bool mine = valid && g == gl;
    unsigned long long mm = __ballot(mine);
    unsigned long long mn = mine ? vmin : ~0ull;
    unsigned long long sm = mine ? vadd : 0ull;
    for (int o = 32; o > 0; o >>= 1) {
      mn = umin64(mn, __shfl_xor(mn, o));
      sm += __shfl_xor(sm, o);
    }
    if (lane == leader) {
      atomicMin(&s_min[gl], mn);
      if (psum) atomicAdd(&s_sum[gl], sm);
    }
    mask &= ~mm;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nf; t += blockDim.x) {
    pmin[(size_t)blockIdx.x * nf + t] = s_min[t];
    if (psum) psum[(size_t)blockIdx.x * nf + t] = s_sum[t];
  }
}

// one block per group: fold the per-block partials of group blockIdx.x;
// which = 0 -> dt_1 and the V~ sum, which = 1 -> dt.  The time step is the
// minimum of the particle terms and the cap dt_max.
__global__ __launch_bounds__(BLOCK) void k_group_reduce(const unsigned long long *__restrict__ pmin,
                                                        const unsigned long long *__restrict__ psum,
                                                        int nblk, int nf, double dt_max, Group *grp,
                                                        int which) {
  __shared__ unsigned long long smn[BLOCK / 64], ssm[BLOCK / 64];
  const int g = blockIdx.x;
  unsigned long long mn = ~0ull, sm = 0ull;
  for (int b = threadIdx.x; b < nblk; b += BLOCK) {
    mn = umin64(mn, pmin[(size_t)b * nf + g]);
    if (psum) sm += psum[(size_t)b * nf + g];
  }
  for (int o = 32; o > 0; o >>= 1) {
    mn = umin64(mn, __shfl_xor(mn, o));
    sm += __shfl_xor(sm, o);
  }
  const int w = threadIdx.x >> 6;
  if (__lane_id() == 0) {
    smn[w] = mn;
    ssm[w] = sm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < BLOCK / 64; ++q) {
      mn = umin64(mn, smn[q]);
      sm += ssm[q];
    }
    mn = umin64(mn, dbits(dt_max));
    if (which == 0) {
      grp[g].dt1_bits = mn;
      grp[g].vsum = sm;
    } else {
      grp[g].dt_bits = mn;
    }
  }
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// ---------------------------------------------------------------------------
// cell hashing and counting sort
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(BLOCK) void k_hash_count(Geom g, Grid G, Parts s, int n,
                                                      uint32_t *__restrict__ cell,
                                                      uint32_t *__restrict__ rank,
                                                      uint32_t *__restrict__ cnt) {
  int i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= n) return;
  double p[3] = {s.x[0][i], s.x[1][i], D == 3 ? s.x[2][i] : 0.0};
  s.h[i] = h_target<D>(g, p);
  int c0 = cell_coord(G, 0, p[0]);
  int c1 = cell_coord(G, 1, p[1]);
  int c2 = D == 3 ? cell_coord(G, 2, p[2]) : 0;
  uint32_t c = ((uint32_t)c2 * (uint32_t)G.nc[1] + (uint32_t)c1) * (uint32_t)G.nc[0] + (uint32_t)c0;
  cell[i] = c;
  rank[i] = atomicAdd(&cnt[c], 1u);
}

constexpr int SCAN_PER = 16;
constexpr int SCAN_TILE = BLOCK * SCAN_PER;

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *lds, uint32_t &total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t x = v;
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) lds[wid] = x;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
  for (int w = 0; w < BLOCK / 64; ++w) {
    uint32_t t = lds[w];
    if (w < wid) pre += t;
    tot += t;
  }
  __syncthreads();
  total = tot;
  return pre + x - v;
}

// out[i] = exclusive prefix of in[] inside its tile; aux[tile] = tile total
__global__ __launch_bounds__(BLOCK) void k_scan_local(const uint32_t *__restrict__ in,
                                                      uint32_t *__restrict__ out,
                                                      uint32_t *__restrict__ aux, uint32_t n) {
  __shared__ uint32_t lds[BLOCK / 64];
  size_t base = (size_t)blockIdx.x * SCAN_TILE + (size_t)threadIdx.x * SCAN_PER;
  uint32_t v[SCAN_PER];
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < SCAN_PER; ++k) {
    size_t idx = base + k;
    v[k] = idx < n ? in[idx] : 0u;
    sum += v[k];
  }
  uint32_t tot;
  uint32_t ex = block_exclusive_scan(sum, lds, tot);
#pragma unroll
  for (int k = 0; k < SCAN_PER; ++k) {
    size_t idx = base + k;
    if (idx < n) out[idx] = ex;
    ex += v[k];
  }
  if (threadIdx.x == 0) aux[blockIdx.x] = tot;
}

// one block: exclusive scan of the tile totals in place (m <= SCAN_TILE)
__global__ __launch_bounds__(BLOCK) void k_scan_top(uint32_t *__restrict__ aux, uint32_t m,
                                                    uint32_t *__restrict__ total_out) {
  __shared__ uint32_t lds[BLOCK / 64];
  size_t base = (size_t)threadIdx.x * SCAN_PER;
  uint32_t v[SCAN_PER];
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < SCAN_PER; ++k) {
    size_t idx = base + k;
    v[k] = idx < m ? aux[idx] : 0u;
    sum += v[k];
  }
  uint32_t tot;
  uint32_t ex = block_exclusive_scan(sum, lds, tot);
#pragma unroll
  for (int k = 0; k < SCAN_PER; ++k) {
    size_t idx = base + k;
    if (idx < m) aux[idx] = ex;
    ex += v[k];
  }
  if (threadIdx.x == 0) *total_out = tot;
}

// out[i] += aux[tile of i]; out[n] = grand total
__global__ __launch_bounds__(BLOCK) void k_scan_add(uint32_t *__restrict__ out,
                                                    const uint32_t *__restrict__ aux, uint32_t n,
                                                    const uint32_t *__restrict__ total) {
  size_t i = (size_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i < n) out[i] += aux[i / SCAN_TILE];
  if (i == 0) out[n] = *total;
}

__global__ __launch_bounds__(BLOCK) void k_scatter(int n, const uint32_t *__restrict__ cell,
                                                   const uint32_t *__restrict__ rank,
                                                   const uint32_t *__restrict__ cstart,
                                                   const uint32_t *__restrict__ oid,
                                                   uint32_t *__restrict__ psrc,
                                                   uint32_t *__restrict__ pkey) {
  int i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= n) return;
  uint32_t pos = cstart[cell[i]] + rank[i];
  if (pos >= (uint32_t)n) return;   // counts are consistent by construction
  psrc[pos] = (uint32_t)i;
  pkey[pos] = oid[i];
}

// insertion sort of one cell's entries by caller id; clears the cell count
__global__ __launch_bounds__(BLOCK) void k_cellsort(uint32_t ncell, const uint32_t *__restrict__ cstart,
                                                    uint32_t *__restrict__ pkey,
                                                    uint32_t *__restrict__ psrc,
                                                    uint32_t *__restrict__ cnt) {
  uint32_t c = blockIdx.x * BLOCK + threadIdx.x;
  if (c >= ncell) return;
  uint32_t b = cstart[c], e = cstart[c + 1];
  cnt[c] = 0u;
  for (uint32_t i = b + 1; i < e; ++i) {
    uint32_t key = pkey[i], src = psrc[i];
    uint32_t j = i;
    while (j > b && pkey[j - 1] > key) {
      pkey[j] = pkey[j - 1];
      psrc[j] = psrc[j - 1];
      --j;
    }
    pkey[j] = key;
    psrc[j] = src;
  }
}

template <int D>
__global__ __launch_bounds__(BLOCK) void k_gather(int n, const uint32_t *__restrict__ psrc, Parts a,
                                                  Parts b) {
  int k = blockIdx.x * BLOCK + threadIdx.x;
  if (k >= n) return;
  uint32_t s = psrc[k];
  if (s >= (uint32_t)n) return;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    b.x[d][k] = a.x[d][s];
    b.v[d][k] = a.v[d][s];
  }
  b.h[k] = a.h[s];
  b.f[k] = a.f[s];
  b.oid[k] = a.oid[s];
}

// ---------------------------------------------------------------------------
// neighbour list (Algorithm 1 "construct Verlet neighbor list")
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(BLOCK) void k_neighbors(Geom g, Grid G, Parts s, int n,
                                                     const uint32_t *__restrict__ cstart,
                                                     const int8_t *__restrict__ rel,
                                                     const Feat *__restrict__ feat,
                                                     const Group *__restrict__ grp, int all,
                                                     uint32_t *__restrict__ nbr,
                                                     uint32_t *__restrict__ nnb, int cap,
                                                     Status *st,
                                                     unsigned long long *__restrict__ pcount) {
  __shared__ unsigned long long s_cnt[BLOCK / 64];
  int i = blockIdx.x * BLOCK + threadIdx.x;
  unsigned long long mine = 0;
  if (i < n) {
    int fi = s.f[i];
    bool want = feat[fi].type != T_SI && (all || grp[fi].active);
    uint32_t count = 0;
    if (want) {
      double xi[3] = {s.x[0][i], s.x[1][i], D == 3 ? s.x[2][i] : 0.0};
      double hi = s.h[i];
      double R = G.rfac * hi;
      R = R < G.rmax ? R : G.rmax;
      int lo_c[3] = {0, 0, 0}, hi_c[3] = {0, 0, 0};
#pragma unroll
      for (int a = 0; a < D; ++a) {
        lo_c[a] = cell_coord(G, a, xi[a] - R);
        hi_c[a] = cell_coord(G, a, xi[a] + R);
      }
      const int8_t *relrow = rel + fi * g.nf;
      for (int cz = lo_c[2]; cz <= hi_c[2]; ++cz)
        for (int cy = lo_c[1]; cy <= hi_c[1]; ++cy) {
          uint32_t row = ((uint32_t)cz * (uint32_t)G.nc[1] + (uint32_t)cy) * (uint32_t)G.nc[0];
          uint32_t jb = cstart[row + lo_c[0]], je = cstart[row + hi_c[0] + 1];
          for (uint32_t j = jb; j < je; ++j) {
            if ((int)j == i) continue;
            double xj2 = D == 3 ? s.x[2][j] : 0.0;
            if (!within<D>(xi, s.x[0][j], s.x[1][j], xj2, hi, s.h[j])) continue;
            int r = relrow[s.f[j]];
            if (!r) continue;
            if ((int)count < cap) nbr[(size_t)count * n + i] = j | (r == 2 ? 0x80000000u : 0u);
            ++count;
          }
        }
      if ((int)count > cap) {
        atomicMax(&st->overflow_max, count);
        atomicExch(&st->overflow, 1u);
        count = cap;
      }
    }
    nnb[i] = count;
    mine = count;
  }
  if (pcount) {
    unsigned long long tot = wave_sum_u64(mine);
    if (__lane_id() == 0) s_cnt[threadIdx.x >> 6] = tot;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long b = 0;
      for (int w = 0; w < BLOCK / 64; ++w) b += s_cnt[w];
      pcount[blockIdx.x] = b;
    }
  }
}

// ---------------------------------------------------------------------------
// sweep A: Shepard term, particle volume, pressure force with the
// feature-boundary correction, mapped onto the feature
// ---------------------------------------------------------------------------
template <int D, typename R>
__global__ __launch_bounds__(BLOCK) void k_sweep_a(Geom g, double p0, int bw, Parts s, int n,
                                                   const uint32_t *__restrict__ nbr,
                                                   const uint32_t *__restrict__ nnb,
                                                   const Feat *__restrict__ feat,
                                                   const BNorm *__restrict__ bn, Group *grp,
                                                   R *__restrict__ ap0, R *__restrict__ ap1,
                                                   R *__restrict__ ap2, double *__restrict__ dbg_gam,
                                                   double *__restrict__ dbg_vt,
                                                   unsigned long long *__restrict__ pmin,
                                                   unsigned long long *__restrict__ psum) {
  __shared__ unsigned long long s_min[MAXF], s_sum[MAXF];
  int i = blockIdx.x * BLOCK + threadIdx.x;
  bool act = false;
  int fi = 0;
  unsigned long long dtb = ~0ull, vfix = 0ull;
  if (i < n) {
    fi = s.f[i];
    const Feat F = feat[fi];
    act = F.type != T_SI && grp[fi].active;
    if (act) {
      const int k = F.k;
      double xi[3] = {s.x[0][i], s.x[1][i], D == 3 ? s.x[2][i] : 0.0};
      double vi[3] = {s.v[0][i], s.v[1][i], D == 3 ? s.v[2][i] : 0.0};
      if (grp[fi].reset_now) {
        vi[0] = vi[1] = vi[2] = 0.0;
#pragma unroll
        for (int a = 0; a < D; ++a) s.v[a][i] = 0.0;
      }
      const double hid = s.h[i];
      const R hi = (R)hid;
      const R ihi = rcp_(hi);
      const R alpha = kalpha<R>(k);
      const R hik = powk(hi, k), hi2k = hik * hik;
      const R ihik = powk(ihi, k);
      const R wself = alpha * ihik;
      const R P0 = (R)p0;
      Acc<R> S, gam, Pi[3], B[3];
      S.init(wself);
      gam.init(wself * hik);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        Pi[a].init(R(0));
        B[a].init(R(0));
      }
      const uint32_t cnt = nnb[i];
      for (uint32_t e = 0; e < cnt; ++e) {
        const uint32_t u = nbr[(size_t)e * n + i];
        const uint32_t j = u & 0x7fffffffu;
        R dx[3];
        dx[0] = (R)(xi[0] - s.x[0][j]);
        dx[1] = (R)(xi[1] - s.x[1][j]);
        dx[2] = D == 3 ? (R)(xi[2] - s.x[2][j]) : R(0);
        const R r = sqrt_(dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2]);
        const R hj = (R)s.h[j];
        const R hjk = powk(hj, k), hj2k = hjk * hjk;
        const R ihij = rcp_(R(0.5) * (hi + hj));
        const R qij = r * ihij;
        if (!(u >> 31)) {
          const R w = alpha * wshape(k, r * ihi) * ihik;           // W(r, h_i)
          S.add(w);
          gam.add(w * hjk);
          const R ih2 = ihij * ihij;
          const R ihk2 = k == 1 ? ih2 * ihij : (k == 2 ? ih2 * ih2 : ih2 * ih2 * ihij);
          const R c = P0 * (hi2k + hj2k) * alpha * dwq(k, qij) * ihk2;   // (dW/dr)/r at h_ij
#pragma unroll
          for (int a = 0; a < D; ++a) Pi[a].add(c * dx[a]);
        } else {
          const int fb = s.f[j];
          const BNorm N = bn[fi * g.nf + fb];
          double nv[3];
          if (N.mode == 2) {
            const double *cc = g.hc[N.hole];
            double d0 = cc[0] - s.x[0][j], d1 = cc[1] - s.x[1][j];
            double d2 = D == 3 ? cc[2] - s.x[2][j] : 0.0;
            double il = 1.0 / __builtin_sqrt(d0 * d0 + d1 * d1 + d2 * d2);
            nv[0] = d0 * il;
            nv[1] = d1 * il;
            nv[2] = d2 * il;
          } else {
            nv[0] = N.n[0];
            nv[1] = N.n[1];
            nv[2] = N.n[2];
          }
          const R om = bw == 0 ? rcp_(hj) : (bw == 1 ? powk(hj, k) * rcp_(hj) : R(0));
          const R w = alpha * wshape(k, qij) * powk(ihij, k);      // W(r, h_ib)
          const R c = P0 * (hi2k + hj2k) * w * om;
#pragma unroll
          for (int a = 0; a < D; ++a) B[a].add(c * (R)nv[a]);
        }
      }
      const double gm = (double)gam.get();
      double ap[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int a = 0; a < D; ++a) ap[a] = -(((double)Pi[a].get() + (double)B[a].get()) / gm);
      tangent<D>(g, F, xi, ap);
      ap0[i] = (R)ap[0];
      ap1[i] = (R)ap[1];
      if (D == 3) ap2[i] = (R)ap[2];
      const double vt = 1.0 / (double)S.get();
      if (dbg_gam) dbg_gam[i] = gm;
      if (dbg_vt) dbg_vt[i] = vt;
      // Eq. (fa_time_step_size) terms from a^p and v^n
      const double rc = 2.0 * hid;
      double dt = __builtin_inf();
      double am = __builtin_sqrt(ap[0] * ap[0] + ap[1] * ap[1] + ap[2] * ap[2]);
      if (am > 0.0) dt = 0.25 * __builtin_sqrt(rc / am);
      double vm = __builtin_sqrt(vi[0] * vi[0] + vi[1] * vi[1] + vi[2] * vi[2]);
      if (vm > 0.0) {
        double t = rc / (40.0 * vm);
        dt = t < dt ? t : dt;
      }
      dtb = dbits(dt);
      vfix = (unsigned long long)__builtin_llrint(vt * grp[fi].vscale);
    } else {
      ap0[i] = R(0);
      ap1[i] = R(0);
      if (D == 3) ap2[i] = R(0);
      if (dbg_gam) dbg_gam[i] = 0.0;
      if (dbg_vt) dbg_vt[i] = 0.0;
    }
  }
  block_group_reduce(act, fi, dtb, vfix, s_min, s_sum, g.nf, pmin, psum);
}

// ---------------------------------------------------------------------------
// sweep B: mid-point velocity, viscous force, damping
// ---------------------------------------------------------------------------
template <int D, typename R>
__global__ __launch_bounds__(BLOCK) void k_sweep_b(Geom g, Parts s, int n,
                                                   const uint32_t *__restrict__ nbr,
                                                   const uint32_t *__restrict__ nnb,
                                                   const Feat *__restrict__ feat, Group *grp,
                                                   const R *__restrict__ ap0,
                                                   const R *__restrict__ ap1,
                                                   const R *__restrict__ ap2, R *__restrict__ a0,
                                                   R *__restrict__ a1, R *__restrict__ a2,
                                                   double *__restrict__ dbg_vm0,
                                                   double *__restrict__ dbg_vm1,
                                                   double *__restrict__ dbg_vm2,
                                                   unsigned long long *__restrict__ pmin) {
  __shared__ unsigned long long s_min[MAXF], s_sum[MAXF];
  int i = blockIdx.x * BLOCK + threadIdx.x;
  bool act = false;
  int fi = 0;
  unsigned long long dtb = ~0ull;
  if (i < n) {
    fi = s.f[i];
    const Feat F = feat[fi];
    act = F.type != T_SI && grp[fi].active;
    if (act) {
      const int k = F.k;
      const double dt1 = bitsd(grp[fi].dt1_bits);
      const double half = 0.5 * dt1;
      double xi[3] = {s.x[0][i], s.x[1][i], D == 3 ? s.x[2][i] : 0.0};
      double vi[3] = {s.v[0][i], s.v[1][i], D == 3 ? s.v[2][i] : 0.0};
      double api[3] = {(double)ap0[i], (double)ap1[i], D == 3 ? (double)ap2[i] : 0.0};
      double vti[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) vti[a] = vi[a] + half * api[a];
      const double vmi = __builtin_sqrt(vti[0] * vti[0] + vti[1] * vti[1] + vti[2] * vti[2]);
      const double hid = s.h[i];
      const R hi = (R)hid;
      const R alpha = kalpha<R>(k);
      const R hik = powk(hi, k), hi2k = hik * hik;
      const R etai = (R)(0.2 * hid * vmi) * rcp_(hik);            // eta = rho_t nu, nu = 0.1 r_c |v~|
      const R vtiR[3] = {(R)vti[0], (R)vti[1], (R)vti[2]};
      const R halfR = (R)half;
      Acc<R> Fv[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) Fv[a].init(R(0));
      const uint32_t cnt = nnb[i];
      for (uint32_t e = 0; e < cnt; ++e) {
        const uint32_t u = nbr[(size_t)e * n + i];
        if (u >> 31) continue;
        const uint32_t j = u;
        R dx[3];
        dx[0] = (R)(xi[0] - s.x[0][j]);
        dx[1] = (R)(xi[1] - s.x[1][j]);
        dx[2] = D == 3 ? (R)(xi[2] - s.x[2][j]) : R(0);
        const R r = sqrt_(dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2]);
        const R hj = (R)s.h[j];
        const R hjk = powk(hj, k), hj2k = hjk * hjk;
        R vtj[3];
        vtj[0] = (R)s.v[0][j] + halfR * ap0[j];
        vtj[1] = (R)s.v[1][j] + halfR * ap1[j];
        vtj[2] = D == 3 ? (R)s.v[2][j] + halfR * ap2[j] : R(0);
        const R vmj = sqrt_(vtj[0] * vtj[0] + vtj[1] * vtj[1] + vtj[2] * vtj[2]);
        const R etaj = R(0.2) * hj * vmj * rcp_(hjk);
        const R es = etai + etaj;
        const R H = es > R(0) ? R(2) * etai * etaj * rcp_(es) : R(0);
        const R ihij = rcp_(R(0.5) * (hi + hj));
        const R ih2 = ihij * ihij;
        const R ihk2 = k == 1 ? ih2 * ihij : (k == 2 ? ih2 * ih2 : ih2 * ih2 * ihij);
        const R c = H * (hi2k + hj2k) * alpha * dwq(k, r * ihij) * ihk2;
#pragma unroll
        for (int a = 0; a < D; ++a) Fv[a].add(c * (vtiR[a] - vtj[a]));
      }
      double fv[3] = {(double)Fv[0].get(), (double)Fv[1].get(), D == 3 ? (double)Fv[2].get() : 0.0};
      tangent<D>(g, F, xi, fv);
      const double eps = grp[fi].eps;
      double acc[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) acc[a] = api[a] + fv[a] - eps * vi[a];
      a0[i] = (R)acc[0];
      a1[i] = (R)acc[1];
      if (D == 3) a2[i] = (R)acc[2];
      if (dbg_vm0) {
        dbg_vm0[i] = vti[0];
        dbg_vm1[i] = vti[1];
        if (D == 3) dbg_vm2[i] = vti[2];
      }
      const double rc = 2.0 * hid;
      double dt = __builtin_inf();
      const double am = __builtin_sqrt(acc[0] * acc[0] + acc[1] * acc[1] + acc[2] * acc[2]);
      if (am > 0.0) dt = 0.25 * __builtin_sqrt(rc / am);
      if (vmi > 0.0) {
        double t = rc / (40.0 * vmi);
        dt = t < dt ? t : dt;
      }
      dtb = dbits(dt);
    } else {
      a0[i] = R(0);
      a1[i] = R(0);
      if (D == 3) a2[i] = R(0);
      if (dbg_vm0) {
        dbg_vm0[i] = 0.0;
        dbg_vm1[i] = 0.0;
        if (D == 3) dbg_vm2[i] = 0.0;
      }
    }
  }
  block_group_reduce(act, fi, dtb, 0ull, s_min, s_sum, g.nf, pmin, nullptr);
}

// ---------------------------------------------------------------------------
// integration with feature projection (FP64 in every precision mode)
// ---------------------------------------------------------------------------
template <int D, typename R>
__global__ __launch_bounds__(BLOCK) void k_integrate(Geom g, Parts s, int n,
                                                     const Feat *__restrict__ feat,
                                                     const Group *__restrict__ grp,
                                                     const R *__restrict__ a0,
                                                     const R *__restrict__ a1,
                                                     const R *__restrict__ a2, Status *st,
                                                     unsigned long long *__restrict__ pesc) {
  __shared__ unsigned long long s_esc[BLOCK / 64];
  int i = blockIdx.x * BLOCK + threadIdx.x;
  bool escaped = false;
  if (i < n) {
    const int fi = s.f[i];
    const Feat F = feat[fi];
    if (F.type != T_SI && grp[fi].active) {
      const double dt = bitsd(grp[fi].dt_bits);
      double acc[3] = {(double)a0[i], (double)a1[i], D == 3 ? (double)a2[i] : 0.0};
      double x[3] = {s.x[0][i], s.x[1][i], D == 3 ? s.x[2][i] : 0.0};
      double v[3] = {s.v[0][i], s.v[1][i], D == 3 ? s.v[2][i] : 0.0};
      double vh[3], xs[3] = {0.0, 0.0, 0.0};
      bool finite = true;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        vh[a] = v[a] + 0.5 * dt * acc[a];
        xs[a] = x[a] + dt * vh[a];
        finite = finite && __builtin_isfinite(xs[a]);
      }
      if (!finite) {
        if (atomicExch(&st->nan_flag, 1u) == 0u) st->nan_oid = s.oid[i];
      } else if (F.kind == K_VOL) {
        if (!inside<D>(g, xs)) {
          escaped = true;
#pragma unroll
          for (int a = 0; a < D; ++a) s.v[a][i] = 0.0;
        } else {
          double vn[3];
#pragma unroll
          for (int a = 0; a < D; ++a) {
            vn[a] = vh[a] + 0.5 * dt * acc[a];
            s.x[a][i] = xs[a];
            s.v[a][i] = vn[a];
          }
        }
      } else {
        project<D>(g, F, xs);
        double vn[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int a = 0; a < D; ++a) vn[a] = vh[a] + 0.5 * dt * acc[a];
        tangent<D>(g, F, xs, vn);
#pragma unroll
        for (int a = 0; a < D; ++a) {
          s.x[a][i] = xs[a];
          s.v[a][i] = vn[a];
        }
      }
    }
  }
  unsigned long long m = __ballot(escaped);
  if (__lane_id() == 0) s_esc[threadIdx.x >> 6] = (unsigned long long)__popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long b = 0;
    for (int w = 0; w < BLOCK / 64; ++w) b += s_esc[w];
    pesc[blockIdx.x] = b;
  }
}

// ---------------------------------------------------------------------------
// control of every feature; prepares the next step (one block)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_control(Ctl P, Group *grp, int nf, Status *st,
                                                   const unsigned long long *__restrict__ pcount,
                                                   const unsigned long long *__restrict__ pesc,
                                                   int nblk) {
  __shared__ int moving;
  __shared__ unsigned long long s_c[BLOCK / 64], s_e[BLOCK / 64];
  const int q = threadIdx.x;
  if (q == 0) moving = 0;
  unsigned long long c = 0, e = 0;
  for (int b = q; b < nblk; b += BLOCK) {
    c += pcount[b];
    e += pesc[b];
  }
  c = wave_sum_u64(c);
  e = wave_sum_u64(e);
  if (__lane_id() == 0) {
    s_c[q >> 6] = c;
    s_e[q >> 6] = e;
  }
  __syncthreads();
  if (q < nf) {
    Group &G = grp[q];
    if (G.tracked && G.phase != PH_FROZEN) {
      const double dt1 = bitsd(G.dt1_bits), dt = bitsd(G.dt_bits);
      const double vbar = (double)G.vsum / G.vscale;
      G.dt1 = dt1;
      G.dt = dt;
      control_law(P, G, vbar, dt);
    }
    G.active = G.tracked && G.phase != PH_FROZEN;
    G.reset_now = G.reset_next;
    G.eps = damping(P, G);
    if (G.active) atomicOr(&moving, 1);
  }
  __syncthreads();
  if (q == 0) {
    unsigned long long ct = 0, et = 0;
    for (int w = 0; w < BLOCK / 64; ++w) {
      ct += s_c[w];
      et += s_e[w];
    }
    st->steps += 1ull;
    st->inter_last = ct;
    st->inter_total += ct;
    st->escaped += et;
    st->converged = moving ? 0 : 1;
  }
}

// the control law alone over a synthetic series (test entry point)
__global__ void k_control_replay(Ctl P, int n, const double *__restrict__ vbar,
                                 const double *__restrict__ dt, int32_t *__restrict__ phase,
                                 int32_t *__restrict__ reset, double *__restrict__ esys,
                                 Group *scratch) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  Group &G = *scratch;
  for (int k = 0; k < n; ++k) {
    if (G.phase != PH_FROZEN) control_law(P, G, vbar[k], dt[k]);
    phase[k] = G.phase;
    reset[k] = G.reset_next;
    esys[k] = G.esys;
  }
}

}  // namespace sph
