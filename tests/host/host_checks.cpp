// Host-side checks of the library's planning logic (no device needed):
//   - neighbour lists N(i) and interaction lists I(i) of the tree planner
//     against their definitions, by brute force over all box pairs of a level
//     (N: boxes at most one box away per axis, the box itself included;
//     I: children of the parent's neighbours that are not neighbours);
//   - colour classes are independent sets (no two boxes of a class adjacent);
//   - size classes of the device pool: at least the request, at most 1/8 (or
//     256 bytes) above it, non-decreasing.
// Prints OK and returns 0 when every check holds.
#include "../../paper_1508_01835_amd/csrc/linalg.hpp"
#include "../../paper_1508_01835_amd/csrc/tree.hpp"

#include <cstdio>
#include <random>

using namespace ifmm;

static int check_tree(int d, int L, int64_t n, unsigned seed, bool clustered) {
  std::mt19937_64 g(seed);
  std::uniform_real_distribution<double> u(0.0, 1.0);
  std::vector<uint64_t> keys(n);
  for (auto& k : keys) {
    int c[3] = {0, 0, 0};
    for (int a = 0; a < d; ++a) {
      double x = clustered ? 0.5 + 0.2 * (u(g) - 0.5) * u(g) : u(g);
      x = std::min(std::max(x, 0.0), 0.999999);
      c[a] = (int)(x * (1 << L));
    }
    k = interleave_h(c, d, L);
  }
  std::sort(keys.begin(), keys.end());
  HTree T;
  T.n = n; T.d = d; T.L = L;
  plan_tree(T, keys);
  int bad = 0;
  for (int l = 2; l <= L; ++l) {
    const HLevel& lv = T.lev[l];
    for (int i = 0; i < lv.nb; ++i) {
      std::vector<int> N, I;
      for (int j = 0; j < lv.nb; ++j) {
        bool adj = true, padj = true;
        for (int a = 0; a < d; ++a) {
          const int ci = lv.coords[(size_t)i * d + a], cj = lv.coords[(size_t)j * d + a];
          if (std::abs(ci - cj) > 1) adj = false;
          if (std::abs((ci >> 1) - (cj >> 1)) > 1) padj = false;
        }
        if (adj) N.push_back(j);
        else if (padj) I.push_back(j);
      }
      const std::vector<int> Np(lv.nbr.begin() + lv.nb_start[i], lv.nbr.begin() + lv.nb_start[i + 1]);
      const std::vector<int> Ip(lv.inter.begin() + lv.in_start[i], lv.inter.begin() + lv.in_start[i + 1]);
      if (N != Np || I != Ip) ++bad;
    }
    for (const auto& cls : lv.classes)
      for (size_t x = 0; x < cls.size(); ++x)
        for (size_t y = x + 1; y < cls.size(); ++y)
          if (adjacent(lv, d, cls[x], cls[y])) ++bad;
  }
  if (bad) std::printf("tree d=%d L=%d n=%lld: %d mismatches\n", d, L, (long long)n, bad);
  return bad;
}

int main() {
  int bad = 0;
  unsigned seed = 7;
  for (int d = 1; d <= 3; ++d)
    for (int L = 2; L <= (d == 3 ? 4 : 6); ++L)
      for (int cl = 0; cl < 2; ++cl) bad += check_tree(d, L, d == 1 ? 200 : 3000, seed++, cl == 1);
  size_t prev = 0;
  for (size_t b = 1; b < ((size_t)1 << 34); b = b + b / 7 + 1) {
    const size_t c = DevPool::cls(b);
    if (c < b || c > b + b / 8 + 256 || c < prev) {
      std::printf("pool class of %zu bytes: %zu\n", b, c);
      ++bad;
    }
    prev = c;
  }
  std::printf(bad ? "FAILED %d\n" : "OK\n", bad);
  return bad ? 1 : 0;
}
