// sph_kernels.h -- the gfx950 kernels of one relaxation step.
//
// Per step (Algorithm 1's loop body, every feature at once, all reading x^n);
// h_i = h_t(x_i), the cell of x_i and its rank inside the cell are already
// known from the previous step's integration (or the set-up hash):
//   k_scan           single-pass exclusive scan of the cell counts (decoupled
//                    look-back) -> cell start table
//   k_scatter        position of every particle in cell order
//   k_rank_gather    order inside a cell by caller id (canonical, history
//                    free), permute the particle records into it, and store
//                    the boundary normals of particles on holes
//   k_nbr_forces     ELL neighbour list (exact FP64 predicate + feature
//                    relation) fused with the Shepard gamma, V~, pressure
//                    force with the boundary term and its tangent projection
//                    -> a^p; striped minima of dt_1 and sums of V~
//   k_group_reduce   fold the striped accumulators per feature (dt_1, V~ sum)
//   k_sweep_b        mid-point velocity on the fly, viscous force -> a
//   k_group_reduce   fold the striped minima of dt
//   k_integrate_hash v_{n+1/2}, x_{n+1}, projection / rejection,
//                    then h, cell and rank of every particle for the next step
//   k_control        E_sys, phases, resets, damping of every feature (1 block)
// A launch covers every job of a batch: particles carry a global feature id
// (64 per job slot), every kernel reads its particle's job record, and a
// job's cells occupy their own range of the batch's cell ids, so jobs never
// interact and each job's result is the same alone or in any mix.
#pragma once
#include "sph_device.h"

namespace sph {

__device__ __forceinline__ unsigned long long umin64(unsigned long long a, unsigned long long b) {
  return a < b ? a : b;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// The particle's terms of Eq. (fa_time_step_size) from |a|^2 and |v|^2 (the
// third term can never be the smallest, so it is left out): min(0.25
// sqrt(r_c / |a|), r_c / (40 |v|)), infinite when both vanish.  F32: in
// FP32 (the FP32 modes hold the time steps to 1e-5), unless a square is
// beyond FP32's range, where FP32 would give a time step of 0.
template <bool F32>
__device__ __forceinline__ double step_terms(double rc, double a2, double v2) {
  if constexpr (F32) {
    if (!(a2 < 1e36 && v2 < 1e36)) return step_terms<false>(rc, a2, v2);
    const float rcf = (float)rc, am = __builtin_amdgcn_sqrtf((float)a2),
                vm = __builtin_amdgcn_sqrtf((float)v2);
    float dt = __builtin_inff();
    if (am > 0.0f) dt = 0.25f * __builtin_amdgcn_sqrtf(rcf * __builtin_amdgcn_rcpf(am));
    if (vm > 0.0f) {
      const float t = rcf * __builtin_amdgcn_rcpf(40.0f * vm);
      dt = t < dt ? t : dt;
    }
    return (double)dt;
  } else {
    double dt = __builtin_inf();
    const double am = __builtin_sqrt(a2);
    if (am > 0.0) dt = 0.25 * __builtin_sqrt(rc / am);
    const double vm = __builtin_sqrt(v2);
    if (vm > 0.0) {
      const double t = rc / (40.0 * vm);
      dt = t < dt ? t : dt;
    }
    return dt;
  }
}

// Per-key reduction of one wave: each distinct key (a feature, or a job)
// among the valid lanes is reduced with xor shuffles and committed by one lane
// with a device atomic into one of NSTRIPE copies of the accumulator (chosen
// by wave), so no address sees more than a few dozen atomics per launch.
// Minima of non-negative double bit patterns and integer sums are exact and
// order independent, so the result does not depend on scheduling or on which
// other jobs share the launch.
__device__ __forceinline__ void wave_commit(bool valid, int key, unsigned long long vmin,
                                            unsigned long long vadd, unsigned long long *smin,
                                            unsigned long long *ssum) {
  const int stripe = (int)((blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6)) & (NSTRIPE - 1));
  unsigned long long mask = __ballot(valid);
  const int lane = __lane_id();
  while (mask) {
    const int leader = __ffsll((long long)mask) - 1;
    const int kl = __shfl(key, leader);
    const bool mine = valid && key == kl;
    const unsigned long long mm = __ballot(mine);
    unsigned long long mn = mine ? vmin : ~0ull;
    unsigned long long sm = mine ? vadd : 0ull;
    for (int o = 32; o > 0; o >>= 1) {
      mn = umin64(mn, __shfl_xor(mn, o));
      sm += __shfl_xor(sm, o);
    }
    if (lane == leader) {
      if (smin) atomicMin(&smin[(size_t)kl * NSTRIPE + stripe], mn);
      if (ssum && sm) atomicAdd(&ssum[(size_t)kl * NSTRIPE + stripe], sm);
    }
    mask &= ~mm;
  }
}

// read a striped accumulator word (filled by the previous launch) and reset it
__device__ __forceinline__ unsigned long long take(unsigned long long *p, unsigned long long reset) {
  const unsigned long long v = *p;
  *p = reset;
  return v;
}

static_assert(NSTRIPE == 64, "one stripe per lane");

// One wave per feature slot folds its NSTRIPE stripes (a lane each, one
// memory round trip) and resets them; which = 0 -> dt_1 and the V~ sum,
// which = 1 -> dt.  The time step is the minimum of the particle terms and
// the job's dt_max.
__global__ __launch_bounds__(BLOCK) void k_group_reduce(Batch B, int which) {
  const int lane = __lane_id();
  const int q = (int)(blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6));
  if (q < B.njobs * MAXF && B.grp[q].tracked) {   // uniform per wave
    Group &G = B.grp[q];
    unsigned long long mn = take(B.smin + (size_t)q * NSTRIPE + lane, ~0ull);
    unsigned long long sm = which == 0 ? take(B.ssum + (size_t)q * NSTRIPE + lane, 0ull) : 0ull;
    for (int o = 32; o > 0; o >>= 1) {
      mn = umin64(mn, __shfl_xor(mn, o));
      sm += __shfl_xor(sm, o);
    }
    if (lane == 0) {
      mn = umin64(mn, dbits(B.jobs[q / MAXF].ctl.dt_max));
      if (which == 0) {
        G.dt1_bits = mn;
        G.vsum = sm;
      } else {
        G.dt_bits = mn;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// cell hashing and counting sort
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ void hash_one(const Geom &g, const Grid &G, double4 &xh, uint32_t &cell) {
  double p[3] = {xh.x, xh.y, xh.z};
  xh.w = h_target<D>(g, p);
  const int l = h_level(G, xh.w);
  int c0 = cell_coord(G, l, 0, p[0]);
  int c1 = cell_coord(G, l, 1, p[1]);
  int c2 = D == 3 ? cell_coord(G, l, 2, p[2]) : 0;
  cell = G.cbase + G.lbase[l] +
         cell_row<D>(G, l, (uint32_t)c1, (uint32_t)c2) * (uint32_t)G.nc[l][0] + (uint32_t)c0;
}

// Rank of a particle inside its cell.  Lanes of a wave that hold the same
// cell in consecutive lanes form a run (particles are in cell order, and most
// stay in their cell from one step to the next); the run's first lane
// reserves the whole run with one atomic and the others take consecutive
// ranks, so a wave issues one atomic per distinct run instead of one per
// particle.  Valid lanes are a prefix of the wave.  Ranks only need to be
// distinct: k_rank_gather puts each cell in caller-id order afterwards.
__device__ __forceinline__ uint32_t rank_in_cell(uint32_t c, bool valid, uint32_t *cnt) {
  const int lane = __lane_id();
  const uint32_t prev = __shfl_up(c, 1);
  const bool head = valid && (lane == 0 || prev != c);
  const unsigned long long heads = __ballot(head);
  const int nvalid = __popcll(__ballot(valid));
  const unsigned long long below_eq = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
  const unsigned long long above = heads & ~below_eq;
  const int next = above ? __ffsll((long long)above) - 1 : 64;
  uint32_t base = 0;
  if (head) base = atomicAdd(&cnt[c], (uint32_t)((next < nvalid ? next : nvalid) - lane));
  const unsigned long long mine = heads & below_eq;
  const int my_head = mine ? 63 - __clzll((long long)mine) : 0;
  return __shfl(base, my_head) + (uint32_t)(lane - my_head);
}

// h, cell and rank inside the cell of the particles [i0, i1) (set-up and
// test paths; a step gets them from k_integrate_hash)
template <int D>
__global__ __launch_bounds__(BLOCK) void k_hash(Batch B, Parts s, int i0, int i1,
                                                uint32_t *__restrict__ cell,
                                                uint32_t *__restrict__ rank,
                                                uint32_t *__restrict__ cnt) {
  const int i = i0 + (int)(blockIdx.x * BLOCK + threadIdx.x);
  const bool valid = i < i1;
  uint32_t c = 0;
  if (valid) {
    const uint32_t f = s.f[i];
    const JobDev &J = B.jobs[f / MAXF];
    double4 xh = s.xh[i];
    hash_one<D>(J.g, J.G, xh, c);
    s.xh[i] = xh;
    s.xf[i] = scan_record<D>(xh, f);
    cell[i] = c;
  }
  const uint32_t r = rank_in_cell(c, valid, cnt);
  if (valid) rank[i] = r;
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

// Single-pass exclusive scan (decoupled look-back).  Tiles take ids from a
// ticket in dispatch order, so a tile only ever waits for tiles that have
// already started; each tile publishes {flag, value} in one 64-bit word:
// flag 1 = tile aggregate, flag 2 = inclusive prefix.  Flag and value travel
// in the same atomic word and nothing else is communicated between tiles, so
// relaxed device-scope atomics suffice (a release would write back the L2 of
// the XCD on every tile).  A tile's counts are loaded coalesced and
// transposed through LDS so that each thread scans SCAN_PER consecutive
// cells.  status[] and the ticket are cleared by k_scatter, which runs after
// the scan has finished.
__global__ __launch_bounds__(BLOCK) void k_scan(const uint32_t *__restrict__ in,
                                                uint32_t *__restrict__ out, uint32_t n,
                                                unsigned long long *status, uint32_t *ticket,
                                                uint32_t ntiles, unsigned int *gflags,
                                                const unsigned long long *__restrict__ vstate) {
  // with Verlet candidate lists, particles are re-sorted only when the lists
  // are rebuilt
  if (vstate && !vstate[VS_REBUILD]) return;
  __shared__ uint32_t lds[BLOCK / 64];
  __shared__ uint32_t s_tile, s_prefix;
  // tile in LDS, one padding word per SCAN_PER so that the per-thread reads
  // of SCAN_PER consecutive words hit distinct banks
  __shared__ uint32_t tbuf[SCAN_TILE + SCAN_TILE / SCAN_PER];
  if (threadIdx.x == 0) s_tile = atomicAdd(ticket, 1u);
  __syncthreads();
  const uint32_t tile = s_tile;
  if (tile >= ntiles) {            // stale ticket: report, never wait
    if (threadIdx.x == 0) atomicExch(&gflags[0], 1u);
    return;
  }
  const size_t tbase = (size_t)tile * SCAN_TILE;
#pragma unroll
  for (int k = 0; k < SCAN_PER; ++k) {
    const uint32_t t = (uint32_t)k * BLOCK + threadIdx.x;
    const size_t idx = tbase + t;
    tbuf[t + t / SCAN_PER] = idx < n ? in[idx] : 0u;
  }
  __syncthreads();
  uint32_t v[SCAN_PER];
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < SCAN_PER; ++k) {
    v[k] = tbuf[threadIdx.x * (SCAN_PER + 1) + k];
    sum += v[k];
  }
  uint32_t tot;
  uint32_t ex = block_exclusive_scan(sum, lds, tot);
  if (threadIdx.x < 64) {
    // publish the tile aggregate, then look back with the whole wave: lane l
    // reads tile (base - l); tiles before 0 count as an inclusive prefix 0.
    // Predecessors took their tickets earlier and publish without waiting on
    // later tiles, so the loop ends; the spin bound only turns a broken
    // invariant into an error instead of a hang.
    const int lane = threadIdx.x;
    if (lane == 0)
      __hip_atomic_store(&status[tile], ((tile == 0 ? 2ull : 1ull) << 32) | tot, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    uint32_t prefix = 0;
    int base = (int)tile - 1;
    unsigned spins = 0;
    while (base >= 0) {
      const int p = base - lane;
      unsigned long long w = p >= 0 ? __hip_atomic_load(&status[p], __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT)
                                    : (2ull << 32);
      const unsigned flag = (unsigned)(w >> 32);
      const unsigned long long m2 = __ballot(flag == 2u);
      const unsigned long long m0 = __ballot(flag == 0u);
      const int first2 = m2 ? __ffsll((long long)m2) - 1 : 64;
      const unsigned long long upto = first2 >= 63 ? ~0ull : ((2ull << first2) - 1ull);
      if (m0 & upto) {
        if (++spins > (1u << 22)) {
          if (lane == 0) atomicExch(&gflags[0], 1u);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
        continue;
      }
      unsigned long long part = lane <= first2 ? (unsigned long long)(uint32_t)w : 0ull;
      part = wave_sum_u64(part);
      prefix += (uint32_t)part;
      if (first2 < 64) break;
      base -= 64;
    }
    if (lane == 0) {
      if (tile != 0)
        __hip_atomic_store(&status[tile], (2ull << 32) | (uint32_t)(prefix + tot), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      s_prefix = prefix;
      if ((size_t)(tile + 1) * SCAN_TILE >= n) out[n] = prefix + tot;
    }
  }
  __syncthreads();
  ex += s_prefix;
#pragma unroll
  for (int k = 0; k < SCAN_PER; ++k) {   // back through LDS for coalesced stores
    tbuf[threadIdx.x * (SCAN_PER + 1) + k] = ex;
    ex += v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < SCAN_PER; ++k) {
    const uint32_t t = (uint32_t)k * BLOCK + threadIdx.x;
    const size_t idx = tbase + t;
    if (idx < n) out[idx] = tbuf[t + t / SCAN_PER];
  }
}

__global__ __launch_bounds__(BLOCK) void k_scatter(int n, const uint32_t *__restrict__ cell,
                                                   const uint32_t *__restrict__ rank,
                                                   const uint32_t *__restrict__ cstart,
                                                   const uint32_t *__restrict__ oid,
                                                   uint32_t *__restrict__ psrc,
                                                   uint32_t *__restrict__ pkey,
                                                   unsigned long long *__restrict__ status,
                                                   uint32_t ntiles, uint32_t *__restrict__ ticket,
                                                   const unsigned long long *__restrict__ vstate) {
  if (vstate && !vstate[VS_REBUILD]) return;   // no sort between list builds
  const int i = blockIdx.x * BLOCK + threadIdx.x;
  for (uint32_t t = (uint32_t)i; t < ntiles; t += gridDim.x * BLOCK) status[t] = 0ull;
  if (i == 0) *ticket = 0u;
  if (i >= n) return;
  uint32_t pos = cstart[cell[i]] + rank[i];
  if (pos >= (uint32_t)n) return;   // counts are consistent by construction
  psrc[pos] = (uint32_t)i;
  pkey[pos] = oid[i];
}

// Entry u of a cell (filled in atomic order) finds its rank among the cell's
// caller ids and copies its particle to that slot; the first entry of a cell
// clears the cell's count for the next hash.  With Verlet candidate lists the
// particles live in buffer a between rebuilds: with no rebuild due, every
// particle keeps its slot, clears its cell's count and refreshes its boundary
// normal; at a rebuild the sorted copy goes to b (whose slot also records x
// and h), and the list build copies it back into a.
template <int D>
__global__ __launch_bounds__(BLOCK) void k_rank_gather(Batch B, int n, const uint32_t *__restrict__ psrc,
                                                       const uint32_t *__restrict__ pkey,
                                                       const uint32_t *__restrict__ cell,
                                                       const uint32_t *__restrict__ cstart,
                                                       uint32_t *__restrict__ cnt, Parts a,
                                                       Parts b) {
  const int u = blockIdx.x * BLOCK + threadIdx.x;
  if (u >= n) return;
  const bool sorted = !B.skin_on || B.vstate[VS_REBUILD] != 0ull;
  uint32_t src = (uint32_t)u, dst = (uint32_t)u;
  if (sorted) {
    src = psrc[u];
    if (src >= (uint32_t)n) return;
    const uint32_t c = cell[src];
    const uint32_t lo = cstart[c], hi = cstart[c + 1];
    const uint32_t key = pkey[u];
    uint32_t r = 0;
    for (uint32_t v = lo; v < hi; ++v) r += pkey[v] < key ? 1u : 0u;
    if ((uint32_t)u == lo) cnt[c] = 0u;
    dst = lo + r;
    if (dst >= (uint32_t)n) return;
    b.oid[dst] = key;
  } else {
    cnt[cell[u]] = 0u;
  }
  const double4 xh = a.xh[src];
  const uint32_t f = a.f[src];
  if (sorted) {   // without a re-sort the particle stays where it is, in a
    b.f[dst] = (uint16_t)f;
    b.xh[dst] = xh;
    b.v[dst] = a.v[src];
    b.xf[dst] = scan_record<D>(xh, f);
    if (B.skin_on) B.xref[dst] = xh;
  }
  // the domain's outward normal at a particle of a feature of lower dimension
  // than the domain, for the pressure sweep of the volume particles beside it
  // (computed there, it would hold registers inside the neighbour loop):
  // towards the centre of a disc or ball, against the level set's gradient for
  // an ellipse or ellipsoid, the closest segment's for an imported curve, and
  // for a box face, edge or corner the constant normal of the volume's table
  const Feat F = B.feat[f];
  if (F.k < D) {
    if (F.kind == K_POLY && D == 2) {   // an imported curve: the closest segment's right normal
      const Geom &gg = B.jobs[f / MAXF].g;
      const double x[3] = {xh.x, xh.y, xh.z};
      double q[2], t[2];
      seg_tangent<2>(gg, poly_closest<2>(gg, F.hole, x, q), t);
      B.enrm[dst] = make_double4(t[1], -t[0], 0.0, 0.0);
    } else if (F.kind == K_POLY) {   // a 3D curve on the zero set: towards decreasing
                                      // phi, and its closest segment in w
      const Geom &gg = B.jobs[f / MAXF].g;
      const double x[3] = {xh.x, xh.y, xh.z};
      double q[3], m[3];
      const int k = poly_closest<3>(gg, F.hole, x, q);
      ls_unit<3>(gg, x, m);
      B.enrm[dst] = make_double4(-m[0], -m[1], -m[2], (double)k);
    } else if (F.kind == K_LEVEL) {   // the zero level set: towards decreasing phi
      const double x[3] = {xh.x, xh.y, xh.z};
      double m[3];
      ls_unit<D>(B.jobs[f / MAXF].g, x, m);
      B.enrm[dst] = make_double4(-m[0], -m[1], -m[2], 0.0);
    } else if (F.kind == K_SHELL) {   // the ball domain's sphere: radially outwards
      const double *cc = B.jobs[f / MAXF].g.dc;
      const double d0 = xh.x - cc[0], d1 = xh.y - cc[1], d2 = D == 3 ? xh.z - cc[2] : 0.0;
      const double il = 1.0 / __builtin_sqrt(d0 * d0 + d1 * d1 + d2 * d2);
      B.enrm[dst] = make_double4(d0 * il, d1 * il, d2 * il, 0.0);
    } else if (F.kind == K_HOLE) {
      const Geom &g = B.jobs[f / MAXF].g;
      double4 e;
      if (g.hell[F.hole]) {
        const double x[3] = {xh.x, xh.y, xh.z};
        double m[3] = {0.0, 0.0, 0.0};
        ell_normal<D>(g, F.hole, x, m);
        e = make_double4(-m[0], -m[1], -m[2], 0.0);
      } else {
        const double *cc = g.hc[F.hole];
        const double d0 = cc[0] - xh.x, d1 = cc[1] - xh.y, d2 = D == 3 ? cc[2] - xh.z : 0.0;
        const double il = 1.0 / __builtin_sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        e = make_double4(d0 * il, d1 * il, d2 * il, 0.0);
      }
      B.enrm[dst] = e;
    } else {   // a box face, edge or corner, an imported corner: the table's constant
      const int job = f / MAXF, vol = B.jobs[job].vol;
      if (vol >= 0) {
        const BNorm N = B.bn[(size_t)(job * MAXF + vol) * MAXF + (f & (MAXF - 1))];
        B.enrm[dst] = make_double4(N.n[0], N.n[1], N.n[2], 0.0);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Pair sums of sweep A (Eqs. (gamma_disc_renormSPH), (particle_volume),
// (sph_pressure_force_disc_weighted)) of particle i of intrinsic dimension K
// over its neighbour list.  Pair terms are evaluated in R and accumulated by
// Sum<CMP>: in FP64, or (CMP, R = float) in FP32 with Neumaier compensation.
// ---------------------------------------------------------------------------
template <int D, int K, typename R, bool CMP>
__host__ __device__ __forceinline__ void sweep_a_sums(const Geom &g, const Parts &s,
                                             const double4 *__restrict__ enrm,
                                             const BNorm *__restrict__ bnrow, int bw, double p0,
                                             double klen, double bscale,
                                             const uint32_t *__restrict__ nbr, int n, int i,
                                             uint32_t cnt, const double4 &xi, int fi, bool pair_normals,
                                             double &S, double &gam, double Pi[3], double B[3],
                                             const uint32_t *ring = nullptr, uint32_t ring_len = 0,
                                             uint32_t ring_stride = 0, uint32_t lane = 0,
                                             uint32_t nlanes = 1) {
  // h enters rho_t = h^-k; the kernel is evaluated at the smoothing length
  // klen h (cut-off radius 2 klen h)
  const R hi = (R)xi.w;
  const R kl = (R)klen;
  const R ihi = rcp_((R)(klen * xi.w));
  constexpr R alpha = kalphaK<K, R>();
  const R hik = powK<K>(hi), hi2k = hik * hik;
  const R ihik = powK<K>(ihi);
  const R P0 = (R)p0;
  const R wself = alpha * ihik;
  // with several lanes per particle, lane l sums the batches l, l + nlanes,
  // ... of the list (the self term in lane 0); the caller adds the lanes' sums
  Sum<CMP> aS, aG, aP[3], aB[3];
  aS.init(lane == 0 ? (double)wself : 0.0);
  aG.init(lane == 0 ? (double)(wself * hik) : 0.0);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    aP[a].init(0.0);
    aB[a].init(0.0);
  }
  constexpr int NB = SPH_NBATCH;
  static_assert(NB == 4 || NB == LB, "record batches of 4 or 8 tile a list block");
  // records gathered together: GB of a batch's NB (fewer live registers)
  constexpr int GB = SPH_GBATCH < NB ? SPH_GBATCH : NB;
  static_assert(NB % GB == 0, "gather groups tile a batch");
  // The list's last entries may also sit in the caller's LDS ring (entry e
  // in slot e % ring_len, column stride ring_stride): entries from lbase on
  // are read there, the ones before from the list in memory (whole blocks,
  // as lbase is a multiple of LB).  Either way every entry is read in list
  // order, so the sums are the same.
  uint32_t lbase = cnt;
  if (ring != nullptr) lbase = cnt > ring_len ? (cnt - ring_len + LB - 1) / LB * LB : 0u;
  const uint4 *gl = reinterpret_cast<const uint4 *>(nbr) + (size_t)i * (LB / 4);
  for (uint32_t e0 = NB * lane; e0 < cnt; e0 += NB * nlanes) {
    {
      uint32_t u[NB];
      if (e0 < lbase) {   // NB entries of a block in memory: 16-byte loads
#pragma unroll
        for (int h = 0; h < NB / 4; ++h) {
          const uint4 w = gl[(size_t)(e0 / LB) * n * (LB / 4) + (e0 % LB) / 4 + h];
          u[4 * h] = w.x;
          u[4 * h + 1] = w.y;
          u[4 * h + 2] = w.z;
          u[4 * h + 3] = w.w;
        }
      } else {
#pragma unroll
        for (int q = 0; q < NB; ++q) u[q] = ring[((e0 + q) % ring_len) * ring_stride];
      }
#pragma unroll
      for (int q = 0; q < NB; ++q) u[q] = e0 + q < cnt ? u[q] : 0u;
#pragma unroll
      for (int g0 = 0; g0 < NB; g0 += GB) {
      double4 xr[GB];
#pragma unroll
      for (int q = 0; q < GB; ++q) xr[q] = s.xh[u[g0 + q] & 0x7fffffffu];
#pragma unroll
      for (int qg = 0; qg < GB; ++qg) {
        const int q = g0 + qg;
        if (e0 + q >= cnt) break;
        const double4 xj = xr[qg];
        const R dx0 = (R)(xi.x - xj.x), dx1 = (R)(xi.y - xj.y);
        const R dx2 = D == 3 ? (R)(xi.z - xj.z) : R(0);
        const R rr = sqrt_(dx0 * dx0 + dx1 * dx1 + dx2 * dx2);
        const R hj = (R)xj.w;
        const R hjk = powK<K>(hj);
        const R hsum = hi2k + hjk * hjk;
        const R ihij = rcp_(kl * (R(0.5) * (hi + hj)));
        const R qij = rr * ihij;
        if (!(u[q] >> 31)) {
          const R w = alpha * wshapeK<K>(rr * ihi) * ihik;           // W(r, h_i)
          aS.add(w);
          aG.add(w * hjk);
          const R ih2 = ihij * ihij;
          const R ihk2 = K == 1 ? ih2 * ihij : (K == 2 ? ih2 * ih2 : ih2 * ih2 * ihij);
          const R c = P0 * hsum * alpha * dwqK<K>(qij) * ihk2;       // (dW/dr)/r at h_ij
          aP[0].add(c * dx0);
          aP[1].add(c * dx1);
          if (D == 3) aP[2].add(c * dx2);
        } else {
          // the particle volume (Eq. (particle_volume)) is the inverse of i's
          // number density: the boundary particles that act on i count too
          aS.add(alpha * wshapeK<K>(rr * ihi) * ihik);
          double nv[3];
          if constexpr (K == D) {   // the volume: the domain's normal k_rank_gather stored at b
            const double4 e = enrm[u[q] & 0x7fffffffu];
            nv[0] = e.x;
            nv[1] = e.y;
            nv[2] = e.z;
          } else {
            const int fj = s.f[u[q] & 0x7fffffffu];
            const BNorm N = bnrow[fj & (MAXF - 1)];
            if (D == 3 && N.mode >= 7) continue;   // normal of the pair: the pass below
            if (N.mode >= 2) {   // a curved boundary: the normal k_rank_gather stored
              const double4 e = enrm[u[q] & 0x7fffffffu];
              nv[0] = e.x;
              nv[1] = e.y;
              nv[2] = e.z;
            } else {
              nv[0] = N.n[0];
              nv[1] = N.n[1];
              nv[2] = N.n[2];
            }
          }
          const R om = (bw == 0 ? rcp_(hj) : (bw == 1 ? powK<K>(hj) * rcp_(hj) : R(0))) * (R)bscale;
          const R w = alpha * wshapeK<K>(qij) * powK<K>(ihij);          // W(r, h_ib)
          if constexpr (CMP) {   // FP32 terms: the normal rounded to FP32
            const float c = (float)(P0 * hsum * w * om);
            aB[0].add(c * (float)nv[0]);
            aB[1].add(c * (float)nv[1]);
            if (D == 3) aB[2].add(c * (float)nv[2]);
          } else {
            const double c = (double)(P0 * hsum * w * om);
            aB[0].add(c * nv[0]);
            aB[1].add(c * nv[1]);
            if (D == 3) aB[2].add(c * nv[2]);
          }
        }
      }
      }
    }
  }
  if constexpr (D == 3) {
    // A 3D surface patch at a curve (mode 7) or vertex (8) beside it: the
    // normal is the direction to b within i's tangent plane (i's stored
    // normal removed), at a curve also without the part along b's closest
    // segment, normalised.  Only patch particles of a geometry with imported
    // curves take this pass, which keeps its registers out of the main loop.
    if (pair_normals) {
      const double4 ei = enrm[i];
      for (uint32_t e = lane; e < cnt; e += nlanes) {
        const uint32_t v = nbr[((size_t)(e / LB) * n + i) * LB + e % LB];
        if (!(v >> 31)) continue;
        const uint32_t b = v & 0x7fffffffu;
        const BNorm N = bnrow[s.f[b] & (MAXF - 1)];
        if (N.mode < 7) continue;
        const double4 xj = s.xh[b];
        const R dx0 = (R)(xi.x - xj.x), dx1 = (R)(xi.y - xj.y), dx2 = (R)(xi.z - xj.z);
        const R rr = sqrt_(dx0 * dx0 + dx1 * dx1 + dx2 * dx2);
        double d0 = xj.x - xi.x, d1 = xj.y - xi.y, d2 = xj.z - xi.z;
        const double dm = d0 * ei.x + d1 * ei.y + d2 * ei.z;
        d0 -= dm * ei.x;
        d1 -= dm * ei.y;
        d2 -= dm * ei.z;
        if (N.mode == 7) {
          double t[3];
          seg_tangent<3>(g, (int)enrm[b].w, t);
          const double dt = d0 * t[0] + d1 * t[1] + d2 * t[2];
          d0 -= dt * t[0];
          d1 -= dt * t[1];
          d2 -= dt * t[2];
        }
        const double l = __builtin_sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        const double il = l > 0.0 ? 1.0 / l : 0.0;
        const double nv[3] = {d0 * il, d1 * il, d2 * il};
        const R hj = (R)xj.w;
        const R hjk = powK<K>(hj);
        const R hsum = hi2k + hjk * hjk;
        const R ihij = rcp_(kl * (R(0.5) * (hi + hj)));
        const R om = (bw == 0 ? rcp_(hj) : (bw == 1 ? powK<K>(hj) * rcp_(hj) : R(0))) * (R)bscale;
        const R w = alpha * wshapeK<K>(rr * ihij) * powK<K>(ihij);      // W(r, h_ib)
        if constexpr (CMP) {
          const float c = (float)(P0 * hsum * w * om);
          aB[0].add(c * (float)nv[0]);
          aB[1].add(c * (float)nv[1]);
          aB[2].add(c * (float)nv[2]);
        } else {
          const double c = (double)(P0 * hsum * w * om);
          aB[0].add(c * nv[0]);
          aB[1].add(c * nv[1]);
          aB[2].add(c * nv[2]);
        }
      }
    }
  }
  S = aS.get();
  gam = aG.get();
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    Pi[a] = aP[a].get();
    B[a] = aB[a].get();
  }
}

// Appends the hits among tag[0, NB) (0xffffffff: no hit) to a particle's
// column of the LDS ring (slot k at rc[k * stride], slot = entry mod LR) and
// stores each list block they complete to *wp as two 16-byte writes, while
// the capacity of nblk blocks allows.  With a ring of two blocks or more the
// block a batch completes is still whole after the batch (NB <= LB hits
// reach at most LB - 1 entries into the next block), so the test for a
// store runs once per batch instead of once per hit.
template <int NB, int LR>
__host__ __device__ __forceinline__ void append_hits(const uint32_t (&tag)[NB], uint32_t *rc,
                                                     int stride, uint32_t &count, uint4 *&wp,
                                                     uint32_t wstep, uint32_t nblk) {
  static_assert(NB <= LB && LR % LB == 0, "a batch completes at most one block");
  if constexpr (LR >= 2 * LB) {
    const uint32_t c0 = count;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      if (tag[q] != 0xffffffffu) {
        rc[(count % LR) * stride] = tag[q];
        ++count;
      }
    }
    if (count / LB != c0 / LB && count / LB <= nblk) {
      const uint32_t k0 = (c0 / LB * LB) % LR;
      wp[0] = make_uint4(rc[k0 * stride], rc[(k0 + 1) * stride], rc[(k0 + 2) * stride],
                         rc[(k0 + 3) * stride]);
      wp[1] = make_uint4(rc[(k0 + 4) * stride], rc[(k0 + 5) * stride], rc[(k0 + 6) * stride],
                         rc[(k0 + 7) * stride]);
      wp += wstep;
    }
  } else {
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      if (tag[q] != 0xffffffffu) {
        const uint32_t k = count % LR;
        rc[k * stride] = tag[q];
        ++count;
        if (k % LB == LB - 1 && count / LB <= nblk) {
          const uint32_t k0 = k - (LB - 1);
          wp[0] = make_uint4(rc[k0 * stride], rc[(k0 + 1) * stride], rc[(k0 + 2) * stride],
                             rc[(k0 + 3) * stride]);
          wp[1] = make_uint4(rc[(k0 + 4) * stride], rc[(k0 + 5) * stride], rc[(k0 + 6) * stride],
                             rc[(k0 + 7) * stride]);
          wp += wstep;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// neighbour list (Algorithm 1 "construct Verlet neighbor list") and, in the
// same launch, sweep A over it; FORCES = false builds the lists only (test
// entry point).  The candidate scan covers, for every cell row within R_i of
// x_i, only the cells under the chord of the disc (sphere) of radius R_i, so
// no neighbour is skipped and fewer non-neighbours are tested.  The pair sums
// then run over the list just written, so the force math executes once per
// neighbour instead of once per candidate.  Every particle reads its own
// job's geometry and grid; cells of different jobs never meet.
// ---------------------------------------------------------------------------
// MODE 0: candidates from the cell scan, as above.  MODE 1 (FORCES = false,
// only when a rebuild is due): the Verlet candidate list of every
// non-singular particle, the cell scan at the reach (c + delta) h with the
// FP32 test alone, widened by its error bound so that it keeps every pair
// within that reach.  MODE 2: candidates from the particle's Verlet list
// instead of the cell scan, classified and summed as in MODE 0.
template <int D, typename R, bool FORCES, int NB, bool CMP = false, int MODE = 0, int LPP = 1>
__global__ __launch_bounds__(BLOCK) void k_nbr_forces(
    Batch B, Parts s, const uint32_t *__restrict__ cstart, int all, uint32_t *__restrict__ nbr,
    uint32_t *__restrict__ nnb, typename Vec4<R>::T *__restrict__ ap,
    double *__restrict__ dbg_gam, double *__restrict__ dbg_vt, Parts home) {
  static_assert(MODE == 0 || (MODE == 1 && !FORCES) || MODE == 2, "candidate list modes");
  if (MODE == 1) {
    if (B.vstate[VS_REBUILD] == 0ull) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) B.vstate[VS_BUILDS] += 1ull;
    // s holds the particles just sorted; they go back to the buffer the
    // steps use between rebuilds (no kernel of this launch reads it)
    const int c = xcd_block() * BLOCK + threadIdx.x;
    if (c < B.n) {
      home.xh[c] = s.xh[c];
      home.v[c] = s.v[c];
      home.f[c] = s.f[c];
      home.oid[c] = s.oid[c];
      home.xf[c] = s.xf[c];
    }
  }
  using R4 = typename Vec4<R>::T;
  // hits collect in the thread's own column of an LDS ring of LR entries (a
  // multiple of LB; see the append below); it keeps the last LR entries, so
  // that in the FP32 modes a list no longer than LR stays whole in LDS,
  // where the pair sums read it (the FP64 sums read the list from memory:
  // the ring's addressing would cost them a wave per SIMD); the Verlet build
  // keeps two blocks, so that its block stores are tested once per batch
  constexpr bool LDS_SUMS = FORCES && sizeof(R) == 4;
  constexpr int LR = LDS_SUMS ? SPH_LDS_LIST : (MODE == 1 ? 2 * LB : LB);
  static_assert(LR % LB == 0, "the ring holds whole blocks");
  // LPP lanes per particle (2: the Verlet filter and the sums split between
  // two adjacent lanes, which doubles the waves that hide the gathers'
  // latency); the particle's lanes share its ring column
  static_assert(LPP == 1 || (LPP == 2 && MODE == 2 && LDS_SUMS && LB == 8),
                "two lanes per particle: the Verlet filter with the sums in LDS");
  constexpr int PB = BLOCK / LPP;
  __shared__ uint32_t ring[LR][PB];
  const int col = (int)threadIdx.x / LPP;
  const int lane = (int)threadIdx.x % LPP;
  const int n = B.n;
  const int i = (xcd_block() * BLOCK + (int)threadIdx.x) / LPP;
  bool act = false;
  int fi = 0, job = 0;
  unsigned long long dtb = ~0ull, vfix = 0ull, mine = 0ull;
  if (i < n) {
    fi = s.f[i];
    job = fi / MAXF;
    const JobDev &J = B.jobs[job];
    const Feat F = B.feat[fi];
    const bool moving = F.type != T_SI && B.grp[fi].active;
    const bool want = F.type != T_SI && (all || MODE == 1 || B.grp[fi].active);
    act = FORCES && moving;
    uint32_t count = 0;
    const double4 xi = s.xh[i];
    if (want) {
      const Grid &G = J.G;
      // scan reach: the cut-off radius, or the Verlet list's in MODE 1
      const double ksup = MODE == 1 ? J.ksup_s : J.ksup;
      double Rs = (MODE == 1 ? J.rfac_s : G.rfac) * xi.w;
      const double rmax = MODE == 1 ? J.rmax_s : G.rmax;
      Rs = Rs < rmax ? Rs : rmax;
      const double pc[3] = {xi.x, xi.y, xi.z};
      // cell levels that can hold a neighbour: h is L-Lipschitz, so a
      // neighbour (r < R_i) has |h_j - h_i| <= L R_i (widened for rounding)
      int lv0 = 0, lv1 = G.nlev - 1;
      if (G.nlev > 1) {
        const double dh = G.lip * Rs * (1.0 + 1e-9);
        lv0 = h_level(G, (xi.w - dh) * (1.0 - 1e-12));
        lv1 = h_level(G, (xi.w + dh) * (1.0 + 1e-12));
      }
      // features that bound fi (bit = local feature id); a candidate of fi's
      // own feature interacts as "same", one of a bounding feature of the same
      // job as "boundary".  The scan only visits cells of i's own job, so a
      // candidate's feature slot is in i's job range and its local id is its
      // low 6 bits.
      const unsigned long long accept = B.bmask[fi] | (1ull << (fi & (MAXF - 1)));
      const double kc2 = J.ksup2;   // c^2, c = support radius / h
      const double A4 = kc2 * (xi.w * xi.w);
      // Candidates are classified in FP32 from the scan records (which hold
      // 2h); only those whose distance is within a thin band around the
      // support radius klen H, H = 2 max(h_i, h_j), are decided by the exact FP64
      // predicate.  Bound: a coordinate of a candidate the scan visits is at
      // most Xb in magnitude (the job's box, or |x_i| + 2 R_i + 2 cells), so
      // each rounded coordinate is off by at most 2^-24 Xb and an FP32
      // distance by at most M = sqrt(D) 2^-23 Xb plus a relative 1e-6.  As H
      // is at least 2 h0 (the sizing's smallest h), M is at most a relative
      // M / (2 h0) of H, so the band of relative half-width
      // w = 2e-6 + M / (2 h0) around H covers every such error and the
      // classification always equals the FP64 predicate.  In 3D the
      // candidate's radius carries the feature id in its 6 low mantissa bits
      // (relative error below 2^-17), so the base width there is 2e-5.
      const float4 xif = scan_record<D>(xi, (uint32_t)fi);
      const float Hif = D == 2 ? xif.z : xif.w;
      float Mf;
      {
        double xb = 0.0;
        const double cm = G.cmax;
#pragma unroll
        for (int a = 0; a < D; ++a) {
          const double l = __builtin_fabs(J.g.lo[a]), h = __builtin_fabs(J.g.hi[a]);
          double m = l > h ? l : h;
          const double own = __builtin_fabs(pc[a]) + 2.0 * Rs + 2.0 * cm;
          m = m > own ? m : own;
          xb = xb > m ? xb : m;
        }
        Mf = (float)((D == 3 ? 1.7320508075688772 : 1.4142135623730951) * 0x1p-23 * xb * 1.01);
      }
      // squared band limits: a certain neighbour below H^2 cin, a certain
      // non-neighbour above H^2 cout
      float cin, cout;
      {
        // the support radius is klen H >= 2 klen h0
        const double w = (D == 2 ? 2e-6 : 2e-5) + (double)Mf * J.iband;
        const double kl = MODE == 1 ? 0.5 * J.ksup_s : J.klen;
        const double k2 = kl * kl;
        cin = w < 1.0 ? (float)((1.0 - w) * (1.0 - w) * k2) : -1.0f;
        cout = (float)((1.0 + w) * (1.0 + w) * k2);
      }
      static_assert(NB >= 1 && NB <= 8, "records are padded by 8");
      // hits collect in the thread's own column of the LDS ring (entry-major,
      // so the lanes of a wave hit distinct banks whatever their fill); each
      // block of LB entries is stored as one 32-byte sector when full (and
      // the last once more, partly filled, at the end).  One LDS write per
      // hit replaces a select over LB registers, which every lane would
      // execute whenever any lane of the wave hits.
      static_assert(LB == 8, "the ring is flushed as two 16-byte stores");
      uint4 *wp = reinterpret_cast<uint4 *>(MODE == 1 ? B.skin : nbr) + (size_t)i * (LB / 4);
      const uint32_t wstep = (uint32_t)n * (LB / 4);
      const uint32_t nblk = (uint32_t)(MODE == 1 ? B.skin_cap : B.cap) / LB;   // blocks of capacity
      if constexpr (MODE == 2) {
        // the Verlet list: every pair within the cut-off is on it (its reach
        // covers the displacements since its build), so filtering it with the
        // same predicate gives the list the cell scan would
        const uint32_t ns = B.nsk[i];
        const size_t sstep = (size_t)n * (LB / 4);
        const uint4 *sp = reinterpret_cast<const uint4 *>(B.skin) + (size_t)i * (LB / 4);
        if constexpr (LPP == 2) {
          // of each block of LB candidates the first lane takes the first
          // four and the second lane the last four; a block's hits enter the
          // ring in list order (the first lane's, then the second's), so the
          // list is the one a single lane writes.  Both lanes of a particle
          // run this loop alike (same particle, same count).
          uint4 w = make_uint4(0u, 0u, 0u, 0u);
          if (ns > 0) w = sp[lane];
          for (uint32_t b0 = 0; b0 < ns; b0 += LB) {
            const uint32_t ub[4] = {w.x, w.y, w.z, w.w};
            if (b0 + LB < ns) {   // the next block's entries, loaded ahead
              sp += sstep;
              w = sp[lane];
            }
            const uint32_t e0 = b0 + 4u * (uint32_t)lane;
            float4 xr[4];
            uint32_t jr[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              jr[q] = e0 + q < ns ? (ub[q] & 0x7fffffffu) : (uint32_t)i;
              xr[q] = s.xf[jr[q]];
            }
            uint32_t tag[4], nh = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const bool cand = e0 + q < ns;
              const float ex = xif.x - xr[q].x, ey = xif.y - xr[q].y;
              const float ez = D == 3 ? xif.z - xr[q].z : 0.0f;
              const float d2 = ex * ex + ey * ey + ez * ez;
              const float Hj = D == 2 ? xr[q].z : xr[q].w;
              const float H = __builtin_fmaxf(Hif, Hj);
              const float H2 = H * H;
              const float tin = H2 * cin, tout = H2 * cout;
              bool hit = cand & (d2 < tin);
              if (cand & !(d2 < tin) & !(d2 > tout))   // near the support radius: exact test
                hit = within_a4<D>(xi, A4, kc2, s.xh[jr[q]]);
              tag[q] = hit ? ub[q] : 0xffffffffu;
              nh += hit ? 1u : 0u;
            }
            // the other lane's hits of this block (lanes 2p and 2p + 1 swap)
            const uint32_t nother = (uint32_t)__shfl_xor((int)nh, 1);
            uint32_t k = count + (lane ? nother : 0u);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              if (tag[q] != 0xffffffffu) {
                ring[k % LR][col] = tag[q];
                ++k;
              }
            }
            const uint32_t cnew = count + nh + nother;
            lane_sync();   // the other lane's ring entries are read below
            // at most LB hits per block: at most one list block completes
            if (cnew / LB != count / LB && cnew / LB <= nblk) {
              const uint32_t k0 = (count / LB * LB) % LR + 4u * (uint32_t)lane;
              wp[lane] = make_uint4(ring[k0][col], ring[k0 + 1][col], ring[k0 + 2][col], ring[k0 + 3][col]);
              wp += wstep;
            }
            count = cnew;
          }
        } else {
        uint4 w0 = make_uint4(0u, 0u, 0u, 0u), w1 = w0;
        if (ns > 0) {
          w0 = sp[0];
          w1 = sp[1];
        }
        for (uint32_t b0 = 0; b0 < ns; b0 += LB) {
          const uint32_t ub[LB] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
          if (b0 + LB < ns) {   // the next block's entries, loaded ahead
            sp += sstep;
            w0 = sp[0];
            w1 = sp[1];
          }
#pragma unroll
          for (int hb = 0; hb < LB; hb += NB) {
            float4 xr[NB];
            uint32_t jr[NB];
#pragma unroll
            for (int q = 0; q < NB; ++q) {
              // entries past the count read the particle's own record
              jr[q] = b0 + hb + q < ns ? (ub[hb + q] & 0x7fffffffu) : (uint32_t)i;
              xr[q] = s.xf[jr[q]];
            }
            uint32_t tag[NB];
#pragma unroll
            for (int q = 0; q < NB; ++q) {
              const bool cand = b0 + hb + q < ns;
              const float ex = xif.x - xr[q].x, ey = xif.y - xr[q].y;
              const float ez = D == 3 ? xif.z - xr[q].z : 0.0f;
              const float d2 = ex * ex + ey * ey + ez * ez;
              const float Hj = D == 2 ? xr[q].z : xr[q].w;
              const float H = __builtin_fmaxf(Hif, Hj);
              const float H2 = H * H;
              const float tin = H2 * cin, tout = H2 * cout;
              bool hit = cand & (d2 < tin);
              if (cand & !(d2 < tin) & !(d2 > tout))   // near the support radius: exact test
                hit = within_a4<D>(xi, A4, kc2, s.xh[jr[q]]);
              tag[q] = hit ? ub[hb + q] : 0xffffffffu;
            }
            append_hits<NB, LR>(tag, &ring[0][col], PB, count, wp, wstep, nblk);
          }
        }
        }
      } else
      for (int lv = lv0; lv <= lv1; ++lv) {
        // a level-lv candidate has h_j < hcap[lv], so none beyond
        // c max(h_i, hcap[lv]) is a neighbour
        double Rl = ksup * (xi.w > G.hcap[lv] ? xi.w : G.hcap[lv]) * (1.0 + 1e-9);
        Rl = Rl < Rs ? Rl : Rs;
        const double R2 = Rl * Rl;
        int lo_c[3] = {0, 0, 0}, hi_c[3] = {0, 0, 0};
#pragma unroll
        for (int a = 1; a < D; ++a) {
          lo_c[a] = cell_coord(G, lv, a, pc[a] - Rl);
          hi_c[a] = cell_coord(G, lv, a, pc[a] + Rl);
        }
        // grid values the row loop needs, kept in registers
        const double c0 = G.c[lv][0], inv0 = G.inv_c[lv][0], lo1 = G.lo[1], c1 = G.c[lv][1];
        const double lo2 = D == 3 ? G.lo[2] : 0.0, c2 = D == 3 ? G.c[lv][2] : 0.0;
        const uint32_t nc0 = (uint32_t)G.nc[lv][0];
        const uint32_t cbase = G.cbase + G.lbase[lv];
        const double u0 = (pc[0] - G.lo[0]) * inv0;     // x of i in cell units
        const double top0 = (double)(G.nc[lv][0] - 1);
        for (int cz = lo_c[2]; cz <= hi_c[2]; ++cz) {
          double dz2 = 0.0;
          if (D == 3) {
            const double z0 = lo2 + cz * c2;
            double dz = z0 - pc[2] > pc[2] - (z0 + c2) ? z0 - pc[2] : pc[2] - (z0 + c2);
            dz = dz - 1e-7 * c2;
            dz = dz > 0.0 ? dz : 0.0;
            dz2 = dz * dz;
          }
          for (int cy = lo_c[1]; cy <= hi_c[1]; ++cy) {
            const double y0 = lo1 + cy * c1;
            double dy = y0 - pc[1] > pc[1] - (y0 + c1) ? y0 - pc[1] : pc[1] - (y0 + c1);
            dy = dy - 1e-7 * c1;
            dy = dy > 0.0 ? dy : 0.0;
            const double w2 = R2 - dy * dy - dz2;
            if (w2 < 0.0) continue;
            // half chord of the row; the FP32 square root (error < 2e-7
            // relative) is covered by the 1e-6 relative widening
            const double wx = (double)sqrt_((float)w2) * (1.0 + 1e-6) + 1e-7 * c0;
            const double wu = wx * inv0;
            double t0 = __builtin_floor(u0 - wu), t1 = __builtin_floor(u0 + wu);
            t0 = t0 >= 0.0 ? t0 : 0.0;   // also maps NaN to cell 0
            t1 = t1 >= 0.0 ? t1 : 0.0;
            t0 = t0 < top0 ? t0 : top0;
            t1 = t1 < top0 ? t1 : top0;
            const uint32_t row = cbase + cell_row<D>(G, lv, (uint32_t)cy, (uint32_t)cz) * nc0;
            const uint32_t jb = cstart[row + (uint32_t)t0], je = cstart[row + (uint32_t)t1 + 1];
            // NB candidates per pass: records loaded together (the arrays are
            // padded by 8 past the capacity), the predicate evaluated for all of
            // them without early exits, then the hits appended in order
            for (uint32_t j0 = jb; j0 < je; j0 += NB) {
              const float4 *rp = s.xf + j0;
              float4 xr[NB];
              uint32_t fr[NB];   // job-local feature id of the candidate
  #pragma unroll
              for (int q = 0; q < NB; ++q) {
                xr[q] = rp[q];
                fr[q] = __float_as_uint(xr[q].w) & (MAXF - 1);
              }
              uint32_t tag[NB];
  #pragma unroll
              for (int q = 0; q < NB; ++q) {
                const uint32_t j = j0 + q;
                const bool rel = (accept >> (fr[q] & (MAXF - 1))) & 1ull;
                const bool cand = rel & (j < je) & (j != (uint32_t)i);
                const float ex = xif.x - xr[q].x, ey = xif.y - xr[q].y;
                const float ez = D == 3 ? xif.z - xr[q].z : 0.0f;
                const float d2 = ex * ex + ey * ey + ez * ez;
                const float Hj = D == 2 ? xr[q].z : xr[q].w;
                const float H = __builtin_fmaxf(Hif, Hj);
                const float H2 = H * H;
                const float tin = H2 * cin, tout = H2 * cout;
                bool hit;
                if constexpr (MODE == 1) {   // Verlet list: all that may lie within reach
                  hit = cand & !(d2 > tout);
                } else {
                  hit = cand & (d2 < tin);
                  if (cand & !(d2 < tin) & !(d2 > tout))   // near the support radius: exact test
                    hit = within_a4<D>(xi, A4, kc2, s.xh[j]);
                }
                tag[q] = hit ? (j | (fr[q] == (uint32_t)(fi & (MAXF - 1)) ? 0u : 0x80000000u))
                             : 0xffffffffu;
              }
              append_hits<NB, LR>(tag, &ring[0][col], PB, count, wp, wstep, nblk);
            }
          }
        }
      }
      if (count % LB != 0 && count / LB < nblk) {   // the last, partly filled block
        const uint32_t k0 = (count / LB * LB) % LR;
        if constexpr (LPP == 2) {
          const uint32_t kl = k0 + 4u * (uint32_t)lane;
          wp[lane] = make_uint4(ring[kl][col], ring[kl + 1][col], ring[kl + 2][col], ring[kl + 3][col]);
        } else {
          wp[0] = make_uint4(ring[k0][col], ring[k0 + 1][col], ring[k0 + 2][col],
                             ring[k0 + 3][col]);
          wp[1] = make_uint4(ring[k0 + 4][col], ring[k0 + 5][col], ring[k0 + 6][col],
                             ring[k0 + 7][col]);
        }
      }
      if (MODE == 1 && (int)count > B.skin_cap) {
        atomicMax(&B.st[job].skin_max, count);
        atomicExch(&B.st[job].skin_overflow, 1u);
        count = B.skin_cap;
      } else if (MODE != 1 && (int)count > B.cap) {
        if (lane == 0) {
          atomicMax(&B.st[job].overflow_max, count);
          atomicExch(&B.st[job].overflow, 1u);
        }
        count = B.cap;
      }
    }
    if (FORCES && act) {
      const int k = F.k;
      double4 v4 = s.v[i];
      if (B.grp[fi].reset_now) {
        v4 = make_double4(0.0, 0.0, 0.0, 0.0);
        if (lane == 0) s.v[i] = v4;
      }
      const BNorm *bnrow = B.bn + (size_t)fi * MAXF;
      // a 3D patch of a level set with imported curves: pair-dependent normals
      const bool pairn = D == 3 && F.kind == K_LEVEL && J.g.cpts != nullptr;
      double S, gam, Pi[3], B3[3];
      if (k == D)
        sweep_a_sums<D, D, R, CMP>(J.g, s, B.enrm, bnrow, J.bw, J.p0, J.klen, J.bscale, nbr, n, i, count, xi, fi, pairn, S, gam, Pi, B3,
                                        LDS_SUMS ? &ring[0][col] : nullptr, LR, PB, lane, LPP);
      else if (k == D - 1)
        sweep_a_sums<D, D - 1, R, CMP>(J.g, s, B.enrm, bnrow, J.bw, J.p0, J.klen, J.bscale, nbr, n, i, count, xi, fi, pairn, S, gam, Pi, B3,
                                        LDS_SUMS ? &ring[0][col] : nullptr, LR, PB, lane, LPP);
      else
        sweep_a_sums<D, 1, R, CMP>(J.g, s, B.enrm, bnrow, J.bw, J.p0, J.klen, J.bscale, nbr, n, i, count, xi, fi, pairn, S, gam, Pi, B3,
                                        LDS_SUMS ? &ring[0][col] : nullptr, LR, PB, lane, LPP);
      if constexpr (LPP == 2) {   // both lanes get the same totals (a + b = b + a)
        S += __shfl_xor(S, 1);
        gam += __shfl_xor(gam, 1);
#pragma unroll
        for (int a = 0; a < D; ++a) {
          Pi[a] += __shfl_xor(Pi[a], 1);
          B3[a] += __shfl_xor(B3[a], 1);
        }
      }
      // the FP32 modes store a^p in FP32 and hold V~ and the time steps to
      // 1e-5: FP32 reciprocals and roots suffice there (relative error 2^-23)
      constexpr bool F32 = sizeof(R) == 4;
      double a3[3] = {0.0, 0.0, 0.0};
      const double ig = F32 ? (double)rcp_((float)gam) : 0.0;
#pragma unroll
      for (int a = 0; a < D; ++a) a3[a] = F32 ? -((Pi[a] + B3[a]) * ig) : -((Pi[a] + B3[a]) / gam);
      double xa[3] = {xi.x, xi.y, xi.z};
      tangent<D>(J.g, F, xa, a3);
      // in 2D the record's free slots carry v^n (after any reset) in the
      // sweep precision, so sweep B gathers one record per neighbour less
      R4 o;
      o.x = (R)a3[0];
      o.y = (R)a3[1];
      o.z = D == 2 ? (R)v4.x : (R)a3[2];
      o.w = D == 2 ? (R)v4.y : R(0);
      const double vt = F32 ? (double)rcp_((float)S) : 1.0 / S;
      if (lane == 0) {
        ap[i] = o;
        if (dbg_gam) dbg_gam[i] = gam;
        if (dbg_vt) dbg_vt[i] = vt;
      }
      // Eq. (fa_time_step_size) terms from a^p and v^n
      const double rc = J.ksup * xi.w;
      const double dt = step_terms<F32>(rc, a3[0] * a3[0] + a3[1] * a3[1] + a3[2] * a3[2],
                                        v4.x * v4.x + v4.y * v4.y + v4.z * v4.z);
      dtb = dbits(dt);
      vfix = (unsigned long long)__builtin_llrint(vt * B.grp[fi].vscale);
    } else if (FORCES && lane == 0) {
      R4 z;
      z.x = z.y = z.z = z.w = R(0);
      ap[i] = z;
      if (dbg_gam) dbg_gam[i] = 0.0;
      if (dbg_vt) dbg_vt[i] = 0.0;
    }
    if (MODE == 1) {
      B.nsk[i] = count;
    } else if (lane == 0) {
      nnb[i] = count;
      mine = count;
    }
  }
  if (FORCES) {
    wave_commit(act && lane == 0, fi, dtb, vfix, B.smin, B.ssum);
    wave_commit(i < n && mine != 0ull, job, 0ull, mine, nullptr, B.scnt);
  }
}

// ---------------------------------------------------------------------------
// mid-point velocity of every moving particle, once: v~ = v + dt_1/2 a^p
// (Eq. momentum_equation_discretized's v~) and eta = 0.2 h |v~| / h^k
// (Eq. viscosity_coefficient), in the sweep precision, so that sweep B
// gathers one 16-byte (FP32) record per neighbour instead of v and a^p
// ---------------------------------------------------------------------------
template <int D, typename R>
__global__ __launch_bounds__(BLOCK) void k_midpoint(Batch B, Parts s,
                                                    const typename Vec4<R>::T *__restrict__ ap,
                                                    typename Vec4<R>::T *__restrict__ mid) {
  using R4 = typename Vec4<R>::T;
  const int i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= B.n) return;
  const int fi = s.f[i];
  const Feat F = B.feat[fi];
  R4 o;
  o.x = o.y = o.z = o.w = R(0);
  if (F.type != T_SI && B.grp[fi].active) {
    const R halfR = (R)(0.5 * bitsd(B.grp[fi].dt1_bits));
    const double4 v = s.v[i];
    const R4 a = ap[i];
    o.x = (R)v.x + halfR * a.x;
    o.y = (R)v.y + halfR * a.y;
    o.z = D == 3 ? (R)v.z + halfR * a.z : R(0);
    const R vm = sqrt_(o.x * o.x + o.y * o.y + o.z * o.z);
    const R h = (R)s.xh[i].w;
    const R hk = F.k == 1 ? powK<1>(h) : (F.k == 2 ? powK<2>(h) : powK<3>(h));
    o.w = (R)(0.1 * B.jobs[fi / MAXF].ksup) * h * vm * rcp_(hk);   // eta = rho_t 0.1 r_c |v~|
  }
  mid[i] = o;
}

// ---------------------------------------------------------------------------
// sweep B pair sums: viscous force of Eq. (momentum_equation_discretized)
// with eta = rho_t nu, nu = 0.1 r_c |v~| (Eq. (viscosity_coefficient)), the
// mid-point velocities v~_j = v_j + dt_1/2 a^p_j formed on the fly
// ---------------------------------------------------------------------------
// MID: neighbours' v~ and eta come from their mid-point records (3D);
// otherwise they are formed here from the a^p record, which in 2D also holds
// v (an extra pass for mid-point records costs more than it saves in 2D).
// XF (FP32 sums): a neighbour's position and h come from its 16-byte FP32
// scan record instead of the 32-byte FP64 one, so the pair differences are
// those of FP32-rounded coordinates; in 3D that record's h carries the
// feature id in its 6 low mantissa bits (relative change below 2^-17).  The
// FP64 mode gathers the FP64 record.
template <int D, int K, typename R, bool MID, bool CMP, int NL = 1>
__device__ __forceinline__ void sweep_b_sums(const Parts &s, const typename Vec4<R>::T *__restrict__ ap,
                                             const typename Vec4<R>::T *__restrict__ mid,
                                             const uint32_t *__restrict__ nbr, int n, int i,
                                             uint32_t cnt, const double4 &xi, const double vti[3],
                                             double vmi, double half, double klen, double Fv[3],
                                             int lane = 0) {
  using R4 = typename Vec4<R>::T;
  const R hi = (R)xi.w;
  constexpr R alpha = kalphaK<K, R>();
  const R hik = powK<K>(hi), hi2k = hik * hik;
  const R kl = (R)klen;
  const R nuf = (R)(0.2 * klen);   // nu = 0.1 r_c |v~| = 0.2 klen h |v~|
  const R etai = (R)(0.2 * klen * xi.w * vmi) * rcp_(hik);
  const R vtiR[3] = {(R)vti[0], (R)vti[1], (R)vti[2]};
  const R halfR = (R)half;
  constexpr bool XF = sizeof(R) == 4;
  const float3 xfi = make_float3((float)xi.x, (float)xi.y, (float)xi.z);
  Sum<CMP> aF[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) aF[a].init(0.0);
  constexpr int NB = SPH_NBATCH;
  static_assert(LB % NB == 0, "record batches tile a list block");
  // with NL = 2 lanes per particle, lane l takes entries 4l .. 4l + 3 of
  // every block (the caller adds the lanes' sums)
  static_assert(NL == 1 || (NL == 2 && NB <= 4), "two lanes: a lane's half block in batches");
  constexpr int PER = LB / NL;   // entries of a block per lane
  const uint4 *blk = reinterpret_cast<const uint4 *>(nbr) + (size_t)i * (LB / 4);
  for (uint32_t b0 = 0; b0 < cnt; b0 += LB, blk += (size_t)n * (LB / 4)) {
    uint32_t ub[PER];
    if constexpr (NL == 1) {
      const uint4 w0 = blk[0], w1 = blk[1];
      ub[0] = w0.x; ub[1] = w0.y; ub[2] = w0.z; ub[3] = w0.w;
      ub[4] = w1.x; ub[5] = w1.y; ub[6] = w1.z; ub[7] = w1.w;
    } else {
      const uint4 w = blk[lane];
      ub[0] = w.x; ub[1] = w.y; ub[2] = w.z; ub[3] = w.w;
    }
#pragma unroll
    for (int hb = 0; hb < PER; hb += NB) {
      const uint32_t e0 = b0 + (uint32_t)(PER * lane) + hb;
      uint32_t u[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) u[q] = e0 + q < cnt ? ub[hb + q] : 0x80000000u;
      double4 xr[NB];
      float4 fr[NB];
      R4 mr[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const uint32_t j = u[q] & 0x7fffffffu;   // boundary entries fetch a valid slot, unused
        if constexpr (XF) fr[q] = s.xf[j]; else xr[q] = s.xh[j];
        mr[q] = MID ? mid[j] : ap[j];
      }
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        if (u[q] >> 31) continue;
        R dx0, dx1, dx2, hj;
        if constexpr (XF) {
          dx0 = (R)(xfi.x - fr[q].x);
          dx1 = (R)(xfi.y - fr[q].y);
          dx2 = D == 3 ? (R)(xfi.z - fr[q].z) : R(0);
          hj = (R)(0.5f * (D == 3 ? fr[q].w : fr[q].z));
        } else {
          const double4 xj = xr[q];
          dx0 = (R)(xi.x - xj.x);
          dx1 = (R)(xi.y - xj.y);
          dx2 = D == 3 ? (R)(xi.z - xj.z) : R(0);
          hj = (R)xj.w;
        }
        const R rr = sqrt_(dx0 * dx0 + dx1 * dx1 + dx2 * dx2);
        const R hjk = powK<K>(hj);
        R vtj[3], etaj;
        if (MID) {
          vtj[0] = mr[q].x;
          vtj[1] = mr[q].y;
          vtj[2] = D == 3 ? mr[q].z : R(0);
          etaj = mr[q].w;
        } else {   // 2D: {a^p_x, a^p_y, v_x, v_y} in the sweep precision
          static_assert(MID || D == 2, "the a^p record carries v only in 2D");
          const R4 apj = mr[q];
          vtj[0] = apj.z + halfR * apj.x;
          vtj[1] = apj.w + halfR * apj.y;
          vtj[2] = R(0);
          const R vmj = sqrt_(vtj[0] * vtj[0] + vtj[1] * vtj[1] + vtj[2] * vtj[2]);
          etaj = nuf * hj * vmj * rcp_(hjk);
        }
        const R es = etai + etaj;
        const R H = es > R(0) ? R(2) * etai * etaj * rcp_(es) : R(0);
        const R ihij = rcp_(kl * (R(0.5) * (hi + hj)));
        const R ih2 = ihij * ihij;
        const R ihk2 = K == 1 ? ih2 * ihij : (K == 2 ? ih2 * ih2 : ih2 * ih2 * ihij);
        const R c = H * (hi2k + hjk * hjk) * alpha * dwqK<K>(rr * ihij) * ihk2;
#pragma unroll
        for (int a = 0; a < D; ++a) aF[a].add(c * (vtiR[a] - vtj[a]));
      }
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) Fv[a] = aF[a].get();
}

// ---------------------------------------------------------------------------
// sweep B: mid-point velocity, viscous force, damping
// ---------------------------------------------------------------------------
template <int D, typename R, bool CMP = false, int LPP = 1>
__global__ __launch_bounds__(BLOCK) void k_sweep_b(Batch B, Parts s,
                                                   const uint32_t *__restrict__ nbr,
                                                   const uint32_t *__restrict__ nnb,
                                                   const typename Vec4<R>::T *__restrict__ ap,
                                                   const typename Vec4<R>::T *__restrict__ mid,
                                                   typename Vec4<R>::T *__restrict__ acc,
                                                   double4 *__restrict__ dbg_vm) {
  using R4 = typename Vec4<R>::T;
  // LPP lanes per particle (2: the neighbour sums split between adjacent lanes)
  static_assert(LPP == 1 || LPP == 2, "one or two lanes per particle");
  const int n = B.n;
  const int i = (xcd_block() * BLOCK + (int)threadIdx.x) / LPP;
  const int lane = (int)threadIdx.x % LPP;
  bool act = false;
  int fi = 0;
  unsigned long long dtb = ~0ull;
  if (i < n) {
    fi = s.f[i];
    const Feat F = B.feat[fi];
    act = F.type != T_SI && B.grp[fi].active;
    if (act) {
      const JobDev &J = B.jobs[fi / MAXF];
      const int k = F.k;
      const double dt1 = bitsd(B.grp[fi].dt1_bits);
      const double half = 0.5 * dt1;
      const double4 xi = s.xh[i];
      const double4 v4 = s.v[i];
      const R4 api4 = ap[i];
      const double vi[3] = {v4.x, v4.y, v4.z};
      const double api[3] = {(double)api4.x, (double)api4.y, D == 3 ? (double)api4.z : 0.0};
      double vti[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) vti[a] = vi[a] + half * api[a];
      const double vmi = __builtin_sqrt(vti[0] * vti[0] + vti[1] * vti[1] + vti[2] * vti[2]);
      const uint32_t cnt = nnb[i];
      double fv[3];
      if (k == D)
        sweep_b_sums<D, D, R, D == 3, CMP, LPP>(s, ap, mid, nbr, n, i, cnt, xi, vti, vmi, half, J.klen, fv, lane);
      else if (k == D - 1)
        sweep_b_sums<D, D - 1, R, D == 3, CMP, LPP>(s, ap, mid, nbr, n, i, cnt, xi, vti, vmi, half, J.klen, fv, lane);
      else
        sweep_b_sums<D, 1, R, D == 3, CMP, LPP>(s, ap, mid, nbr, n, i, cnt, xi, vti, vmi, half, J.klen, fv, lane);
      if constexpr (LPP == 2) {   // both lanes get the same totals (a + b = b + a)
#pragma unroll
        for (int a = 0; a < 3; ++a) fv[a] += __shfl_xor(fv[a], 1);
      }
      double xa[3] = {xi.x, xi.y, xi.z};
      tangent<D>(J.g, F, xa, fv);
      const double eps = B.grp[fi].eps;
      double a3[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) a3[a] = api[a] + fv[a] - eps * vi[a];
      R4 o;
      o.x = (R)a3[0];
      o.y = (R)a3[1];
      o.z = (R)a3[2];
      o.w = R(0);
      if (lane == 0) {
        acc[i] = o;
        if (dbg_vm) dbg_vm[i] = make_double4(vti[0], vti[1], vti[2], 0.0);
      }
      const double rc = J.ksup * xi.w;
      const double dt = step_terms<sizeof(R) == 4>(rc, a3[0] * a3[0] + a3[1] * a3[1] + a3[2] * a3[2],
                                                   vmi * vmi);
      dtb = dbits(dt);
    } else if (lane == 0) {
      R4 z;
      z.x = z.y = z.z = z.w = R(0);
      acc[i] = z;
      if (dbg_vm) dbg_vm[i] = make_double4(0.0, 0.0, 0.0, 0.0);
    }
  }
  wave_commit(act && lane == 0, fi, dtb, 0ull, B.smin, nullptr);
}

// ---------------------------------------------------------------------------
// control of every feature of every job; prepares the next step (one block)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_control(Batch B) {
  __shared__ int moving[MAXJ];
  for (int j = threadIdx.x; j < MAXJ; j += BLOCK) moving[j] = 0;
  __syncthreads();
  for (int q = threadIdx.x; q < B.njobs * MAXF; q += BLOCK) {
    Group &Gq = B.grp[q];
    if (!Gq.tracked) continue;
    const Ctl &P = B.jobs[q / MAXF].ctl;
    if (Gq.phase != PH_FROZEN) {
      const double dt1 = bitsd(Gq.dt1_bits), dt = bitsd(Gq.dt_bits);
      const double vbar = (double)Gq.vsum / Gq.vscale;
      Gq.dt1 = dt1;
      Gq.dt = dt;
      control_law(P, Gq, vbar, dt);
    }
    Gq.active = Gq.phase != PH_FROZEN;
    Gq.reset_now = Gq.reset_next;
    Gq.eps = damping(P, Gq);
    if (Gq.active) atomicOr(&moving[q / MAXF], 1);
  }
  __syncthreads();
  // per job: fold the interaction and escape stripes (a wave per job)
  const int lane = __lane_id();
  for (int j = threadIdx.x >> 6; j < B.njobs; j += BLOCK / 64) {
    unsigned long long c = take(B.scnt + (size_t)j * NSTRIPE + lane, 0ull);
    unsigned long long e = take(B.sesc + (size_t)j * NSTRIPE + lane, 0ull);
    c = wave_sum_u64(c);
    e = wave_sum_u64(e);
    JobStat &S = B.st[j];
    if (lane == 0 && S.live) {
      if (!S.converged) S.steps += 1ull;     // a converged job stops counting
      S.inter_last = c;
      S.inter_total += c;
      S.escaped += e;
      S.converged = moving[j] ? 0 : 1;
    }
  }
  // Verlet lists: rebuild before the next step once some particle has moved
  // as far as its list's reach allows
  if (B.skin_on && threadIdx.x == 0) {
    B.vstate[VS_REBUILD] = B.vstate[VS_TRIP];
    B.vstate[VS_TRIP] = 0ull;
  }
}

// ---------------------------------------------------------------------------
// integration with feature projection (FP64 in every precision mode), then
// h, cell and rank of every particle for the next step's sort
// ---------------------------------------------------------------------------
template <int D, typename R>
__global__ __launch_bounds__(BLOCK) void k_integrate_hash(
    Batch B, Parts s, const typename Vec4<R>::T *__restrict__ acc,
    uint32_t *__restrict__ cell, uint32_t *__restrict__ rank, uint32_t *__restrict__ cnt) {
  const int n = B.n;
  const int i = blockIdx.x * BLOCK + threadIdx.x;
  bool escaped = false;
  int job = 0;
  uint32_t cc = 0;
  double moved = 0.0;
  if (i < n) {
    const int fi = s.f[i];
    job = fi / MAXF;
    const JobDev &J = B.jobs[job];
    const Feat F = B.feat[fi];
    double4 xh = s.xh[i];
    double4 v4 = s.v[i];
    if (F.type != T_SI && B.grp[fi].active) {
      const double dt = bitsd(B.grp[fi].dt_bits);
      const auto a4 = acc[i];
      const double a3[3] = {(double)a4.x, (double)a4.y, (double)a4.z};
      const double x[3] = {xh.x, xh.y, xh.z};
      const double v[3] = {v4.x, v4.y, v4.z};
      double vh[3] = {0.0, 0.0, 0.0}, xs[3] = {0.0, 0.0, 0.0};
      bool finite = true;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        vh[a] = v[a] + 0.5 * dt * a3[a];
        xs[a] = x[a] + dt * vh[a];
        finite = finite && __builtin_isfinite(xs[a]);
      }
      if (!finite) {
        if (atomicExch(&B.st[job].nan_flag, 1u) == 0u) B.st[job].nan_oid = s.oid[i];
      } else if (F.kind == K_VOL && !inside<D>(J.g, xs)) {
        escaped = true;                                   // rejected move: stay, stop
        v4 = make_double4(0.0, 0.0, 0.0, 0.0);
      } else {
        if (F.kind != K_VOL) project<D>(J.g, F, xs);
        // the velocity carried into the next step is v^{n+1/2}, tangent to
        // the feature at x^{n+1}: Algorithm 1 updates the predicted velocity
        // and the position, and no velocity after them
        double vn[3] = {vh[0], vh[1], vh[2]};
        if (F.kind != K_VOL) tangent<D>(J.g, F, xs, vn);
        xh.x = xs[0];
        xh.y = xs[1];
        if (D == 3) xh.z = xs[2];
        v4 = make_double4(vn[0], vn[1], D == 3 ? vn[2] : 0.0, 0.0);
      }
    }
    hash_one<D>(J.g, J.G, xh, cc);
    const float4 rec = scan_record<D>(xh, (uint32_t)fi);
    s.xh[i] = xh;
    s.v[i] = v4;
    s.xf[i] = rec;
    cell[i] = cc;
    if (B.skin_on) {   // displacement since the Verlet list's build, in units of its limit
      const double4 r = B.xref[i];
      const double d0 = xh.x - r.x, d1 = xh.y - r.y, d2 = D == 3 ? xh.z - r.z : 0.0;
      const double d = __builtin_sqrt(d0 * d0 + d1 * d1 + d2 * d2);
      moved = d > 0.0 ? d / (J.move_eps * r.w) : 0.0;
    }
  }
  const uint32_t r = rank_in_cell(cc, i < n, cnt);
  if (i < n) rank[i] = r;
  wave_commit(escaped, job, 0ull, 1ull, nullptr, B.sesc);
  // a wave with a particle past its limit (or non-finite) raises the trip
  // word; every writer stores the same value
  if (B.skin_on && __ballot(!(moved <= 1.0)) && __lane_id() == 0) B.vstate[VS_TRIP] = 1ull;
}

// ---------------------------------------------------------------------------
// the control law alone over a synthetic series (test entry point); state is
// the control state of the one feature replayed, set to a fresh feature's
// (Phase One, no window yet) before the series
__global__ void k_control_replay(Ctl P, int n, const double *__restrict__ vbar,
                                 const double *__restrict__ dt, int32_t *__restrict__ phase,
                                 int32_t *__restrict__ reset, double *__restrict__ esys,
                                 Group *state) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  Group &G = *state;
  {
    Group g0;
    unsigned char *z = reinterpret_cast<unsigned char *>(&g0);
    for (size_t b = 0; b < sizeof g0; ++b) z[b] = 0;
    g0.phase = PH_ONE;
    g0.esys = __builtin_inf();
    g0.tracked = 1;
    G = g0;
  }
  for (int k = 0; k < n; ++k) {
    if (G.phase != PH_FROZEN) control_law(P, G, vbar[k], dt[k]);
    phase[k] = G.phase;
    reset[k] = G.reset_next;
    esys[k] = G.esys;
  }
}

}  // namespace sph
