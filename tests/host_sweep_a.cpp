// Host build of the library's pressure-sweep code (sweep_a_sums and the
// tangent projection of csrc/sph_kernels.h / sph_device.h), for a CPU test
// under AddressSanitizer and UndefinedBehaviorSanitizer: the same functions
// the neighbour kernel runs, fed neighbour lists computed by the oracle, so
// that their results can be compared with the oracle's on the CPU.
//
// Input file (raw, native endianness):
//   int32 D, n, m, n_holes
//   double lo[3], hi[3], holes[n_holes * 15]
//   double sizing: kind, h0, grad, dcap, point[3]
//   double params: kernel_support, boundary_scale, p0, boundary_weighting
//   double xyz[n * 3]; int32 feature[n]
//   int32 idx[m]; int64 off[m + 1]; int32 ids[off[m]]; int8 rel[off[m]]
// Output file: double ap[m * 3], vt[m], gam[m]
#include "../paper_2003_01061_amd/csrc/sph_mesh.hip"

#include <cstdlib>
#include <fstream>

template <typename T>
static void get(std::ifstream &in, T *p, size_t n) {
  in.read(reinterpret_cast<char *>(p), (std::streamsize)(sizeof(T) * n));
  if (!in) {
    std::fprintf(stderr, "short input\n");
    std::exit(2);
  }
}

int main(int argc, char **argv) {
  if (argc != 3 && argc != 4) return 2;
  const uint32_t lanes = argc == 4 ? (uint32_t)std::atoi(argv[3]) : 1u;   // lanes per particle
  if (lanes < 1 || lanes > 2) return 2;
  std::ifstream in(argv[1], std::ios::binary);
  int32_t hdr[4];
  get(in, hdr, 4);
  const int D = hdr[0], n = hdr[1], m = hdr[2], nh = hdr[3];
  std::vector<double> holes((size_t)nh * 15);
  sph_geometry g{};
  g.dim = D;
  get(in, g.lo, 3);
  get(in, g.hi, 3);
  get(in, holes.data(), holes.size());
  g.n_holes = nh;
  g.holes = holes.data();
  double sz[7], pp[4];
  get(in, sz, 7);
  get(in, pp, 4);
  sph_sizing s{};
  s.kind = (int32_t)sz[0];
  s.h0 = sz[1];
  s.grad = sz[2];
  s.dcap = sz[3];
  for (int a = 0; a < 3; ++a) s.point[a] = sz[4 + a];
  sph_params p{};
  p.kernel_support = pp[0];
  p.boundary_scale = pp[1];
  p.p0 = pp[2];
  p.boundary_weighting = (int32_t)pp[3];
  p.window_samples = 10;
  p.sample_every = 20;
  p.reset_period = 100;
  p.ramp_halving = 20;
  p.ramp_steps = 140;
  p.phase2_steps = 400;
  p.max_phase1_steps = 1 << 30;
  p.dt_max = 1.0;
  p.tol = 5e-6;
  std::vector<double> xyz((size_t)n * 3);
  std::vector<int32_t> feat(n), idx(m);
  get(in, xyz.data(), xyz.size());
  get(in, feat.data(), feat.size());
  get(in, idx.data(), idx.size());
  std::vector<int64_t> off((size_t)m + 1);
  get(in, off.data(), off.size());
  std::vector<int32_t> ids(off[m]);
  std::vector<int8_t> rel(off[m]);
  get(in, ids.data(), ids.size());
  get(in, rel.data(), rel.size());
  if (sph_status st = validate(&g, &s, &p)) {
    std::fprintf(stderr, "invalid problem: %s\n", g_err.c_str());
    return 2;
  }

  HostJob J;
  fill_job(J, &g, &s, &p, 0, n);
  const Geom &G = J.dev.g;
  const int nf = J.nf;
  // feature and boundary-normal tables as sph_batch_add builds them (job slot 0)
  std::vector<Feat> hf(MAXF);
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
    for (int j = 0; j < nf; ++j) hb[(size_t)i * MAXF + j] = boundary_normal(D, F, J.feats[j]);
  }
  // particle records in the caller's order (slot = caller id), h from h_t;
  // padded by 8 records as on the device
  std::vector<double4> xh((size_t)n + 8), enrm((size_t)n + 8);
  std::vector<uint16_t> f16((size_t)n + 8, 0);
  for (int i = 0; i < n; ++i) {
    double x[3] = {xyz[3 * (size_t)i], xyz[3 * (size_t)i + 1], D == 3 ? xyz[3 * (size_t)i + 2] : 0.0};
    const double h = D == 2 ? h_target<2>(G, x) : h_target<3>(G, x);
    xh[i] = make_double4(x[0], x[1], x[2], h);
    f16[i] = (uint16_t)feat[i];
    enrm[i] = make_double4(0.0, 0.0, 0.0, 0.0);
    const Feat &F = hf[feat[i]];
    if (F.kind == K_HOLE) {   // the normal out of the domain, as the sort stores it
      if (G.hell[F.hole]) {
        double mv[3] = {0.0, 0.0, 0.0};
        if (D == 2) ell_normal<2>(G, F.hole, x, mv); else ell_normal<3>(G, F.hole, x, mv);
        enrm[i] = make_double4(-mv[0], -mv[1], -mv[2], 0.0);
      } else {
        const double *cc = G.hc[F.hole];
        const double d0 = cc[0] - x[0], d1 = cc[1] - x[1], d2 = D == 3 ? cc[2] - x[2] : 0.0;
        const double il = 1.0 / std::sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        enrm[i] = make_double4(d0 * il, d1 * il, d2 * il, 0.0);
      }
    } else if (F.k < D) {   // a box face, edge or corner: the volume's constant normal
      int vol = -1;
      for (int q = 0; q < nf && vol < 0; ++q)
        if (hf[q].kind == K_VOL) vol = q;
      if (vol >= 0) {
        const BNorm &N = hb[(size_t)vol * MAXF + feat[i]];
        enrm[i] = make_double4(N.n[0], N.n[1], N.n[2], 0.0);
      }
    }
  }
  Parts P{};
  P.xh = xh.data();
  P.f = f16.data();
  // blocked ELL list of the sampled particles: entries 8b..8b+7 of slot i in
  // block b * n + i, the top bit marking a boundary neighbour
  int64_t maxc = 0;
  for (int t = 0; t < m; ++t) maxc = std::max<int64_t>(maxc, off[t + 1] - off[t]);
  const int64_t nblk = (maxc + LB - 1) / LB;
  std::vector<uint32_t> nbr((size_t)(nblk > 0 ? nblk : 1) * n * LB, 0u);
  for (int t = 0; t < m; ++t) {
    const int i = idx[t];
    for (int64_t e = off[t]; e < off[t + 1]; ++e) {
      const int64_t k = e - off[t];
      nbr[((size_t)(k / LB) * n + i) * LB + (size_t)(k % LB)] =
          (uint32_t)ids[e] | (rel[e] == 2 ? 0x80000000u : 0u);
    }
  }
  std::vector<double> out((size_t)m * 5, 0.0);
  for (int t = 0; t < m; ++t) {
    const int i = idx[t];
    const int fi = feat[i];
    const Feat F = hf[fi];
    if (F.type == T_SI) continue;
    const BNorm *bnrow = hb.data() + (size_t)fi * MAXF;
    const uint32_t cnt = (uint32_t)(off[t + 1] - off[t]);
    double S = 0.0, gam = 0.0, Pi[3] = {0.0, 0.0, 0.0}, B3[3] = {0.0, 0.0, 0.0};
    const JobDev &JD = J.dev;
    const bool pairn = D == 3 && F.kind == K_LEVEL && G.cpts != nullptr;
    // the list split over `lanes` lanes as the kernel's lanes of one particle
    // split it, their sums added
    for (uint32_t l = 0; l < lanes; ++l) {
      double s1, g1, p1[3], b1[3];
      if (D == 3) {
        if (F.k == 3)
          sweep_a_sums<3, 3, double, false>(G, P, enrm.data(), bnrow, JD.bw, JD.p0, JD.klen, JD.bscale, nbr.data(), n, i, cnt, xh[i], fi, pairn, s1, g1, p1, b1, nullptr, 0, 0, l, lanes);
        else if (F.k == 2)
          sweep_a_sums<3, 2, double, false>(G, P, enrm.data(), bnrow, JD.bw, JD.p0, JD.klen, JD.bscale, nbr.data(), n, i, cnt, xh[i], fi, pairn, s1, g1, p1, b1, nullptr, 0, 0, l, lanes);
        else
          sweep_a_sums<3, 1, double, false>(G, P, enrm.data(), bnrow, JD.bw, JD.p0, JD.klen, JD.bscale, nbr.data(), n, i, cnt, xh[i], fi, pairn, s1, g1, p1, b1, nullptr, 0, 0, l, lanes);
      } else {
        if (F.k == 2)
          sweep_a_sums<2, 2, double, false>(G, P, enrm.data(), bnrow, JD.bw, JD.p0, JD.klen, JD.bscale, nbr.data(), n, i, cnt, xh[i], fi, pairn, s1, g1, p1, b1, nullptr, 0, 0, l, lanes);
        else
          sweep_a_sums<2, 1, double, false>(G, P, enrm.data(), bnrow, JD.bw, JD.p0, JD.klen, JD.bscale, nbr.data(), n, i, cnt, xh[i], fi, pairn, s1, g1, p1, b1, nullptr, 0, 0, l, lanes);
      }
      S += s1;
      gam += g1;
      for (int a = 0; a < 3; ++a) {
        Pi[a] += p1[a];
        B3[a] += b1[a];
      }
    }
    double a3[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < D; ++a) a3[a] = -((Pi[a] + B3[a]) / gam);
    double xa[3] = {xh[i].x, xh[i].y, xh[i].z};
    if (D == 3) tangent<3>(G, F, xa, a3); else tangent<2>(G, F, xa, a3);
    for (int a = 0; a < 3; ++a) out[(size_t)t * 3 + a] = a3[a];
    out[(size_t)m * 3 + t] = 1.0 / S;
    out[(size_t)m * 4 + t] = gam;
  }
  std::ofstream o(argv[2], std::ios::binary);
  o.write(reinterpret_cast<const char *>(out.data()), (std::streamsize)(sizeof(double) * out.size()));
  return o ? 0 : 3;
}
