// Host build of the neighbour kernel's hit append (append_hits of
// csrc/sph_kernels.h) for a CPU test under AddressSanitizer and
// UndefinedBehaviorSanitizer: random hit patterns in batches of NB
// candidates through a ring of LR entries into a list of nblk blocks of 8
// (the list buffer sized exactly, so a store past the capacity is reported),
// followed by the kernel's store of the last, partly filled block.  Checks:
// the stored entries are the hits in order, up to the capacity; the ring
// holds the last LR hits (two blocks or more: the pressure sweep reads them
// there); the count is the number of hits.  Prints "ok" and the number of
// patterns, or the first mismatch.
#include "../paper_2003_01061_amd/csrc/sph_mesh.hip"

#include <cstdio>
#include <random>

using namespace sph;

template <int NB, int LR>
static int run(std::mt19937_64 &rng, int trials) {
  const int stride = 3, col = 1;   // the particle's column of a 3-column ring
  for (int t = 0; t < trials; ++t) {
    const int ncand = (int)(rng() % 97);
    const uint32_t nblk = 1 + (uint32_t)(rng() % 8);
    const double p = (double)(rng() % 101) / 100.0;
    std::vector<uint32_t> ring((size_t)LR * stride, 0xdeadbeefu);
    std::vector<uint4> list((size_t)nblk * 2);
    for (auto &w : list) w = make_uint4(0xeeeeeeeeu, 0xeeeeeeeeu, 0xeeeeeeeeu, 0xeeeeeeeeu);
    std::vector<uint32_t> want;
    uint32_t count = 0;
    uint4 *wp = list.data();
    const uint32_t wstep = 2;   // blocks of one particle follow each other here
    std::uniform_real_distribution<double> u(0.0, 1.0);
    for (int c0 = 0; c0 < ncand; c0 += NB) {
      uint32_t tag[NB];
      for (int q = 0; q < NB; ++q) {
        const bool hit = c0 + q < ncand && u(rng) < p;
        tag[q] = hit ? (uint32_t)(c0 + q) | ((rng() & 1) ? 0x80000000u : 0u) : 0xffffffffu;
        if (hit) want.push_back(tag[q]);
      }
      append_hits<NB, LR>(tag, ring.data() + col, stride, count, wp, wstep, nblk);
    }
    if (count % LB != 0 && count / LB < nblk) {   // the kernel's last, partly filled block
      const uint32_t k0 = (count / LB * LB) % LR;
      const uint32_t *rc = ring.data() + col;
      wp[0] = make_uint4(rc[k0 * stride], rc[(k0 + 1) * stride], rc[(k0 + 2) * stride], rc[(k0 + 3) * stride]);
      wp[1] = make_uint4(rc[(k0 + 4) * stride], rc[(k0 + 5) * stride], rc[(k0 + 6) * stride],
                         rc[(k0 + 7) * stride]);
    }
    if (count != want.size()) {
      std::printf("NB %d LR %d trial %d: count %u, want %zu\n", NB, LR, t, count, want.size());
      return 1;
    }
    const uint32_t *got = reinterpret_cast<const uint32_t *>(list.data());
    const size_t stored = std::min<size_t>(count, (size_t)nblk * LB);
    for (size_t e = 0; e < stored; ++e)
      if (got[e] != want[e]) {
        std::printf("NB %d LR %d trial %d: entry %zu is %08x, want %08x\n", NB, LR, t, e, got[e], want[e]);
        return 1;
      }
    if (LR >= 2 * LB)
      for (size_t e = count > (uint32_t)LR ? count - LR : 0; e < count; ++e)
        if (ring[(e % LR) * stride + col] != want[e]) {
          std::printf("NB %d LR %d trial %d: ring entry %zu is %08x, want %08x\n", NB, LR, t, e,
                      ring[(e % LR) * stride + col], want[e]);
          return 1;
        }
  }
  return 0;
}

int main() {
  std::mt19937_64 rng(11);
  const int T = 4000;
  int bad = run<2, 8>(rng, T) + run<4, 8>(rng, T) + run<8, 8>(rng, T) + run<2, 16>(rng, T) +
            run<4, 16>(rng, T) + run<8, 16>(rng, T) + run<4, 32>(rng, T) + run<8, 32>(rng, T);
  if (bad) return 1;
  std::printf("ok %d\n", 8 * T);
  return 0;
}
