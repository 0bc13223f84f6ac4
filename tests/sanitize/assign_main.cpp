// Host-sanitizer driver of the library's assignment (Eq. (1) on the reduced
// problem, Sec. 4.3): dense instances large enough for the epsilon-scaled
// auction (the largest with its searches on several threads), its optimality
// certificate and the KD-trees and heaps around them, plus small ones for the shortest-path branch and the reductions.
// Built with AddressSanitizer and UndefinedBehaviorSanitizer on the host
// code only; needs no GPU.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

#include "topsimp.h"

int main() {
  std::mt19937_64 g(7);
  std::normal_distribution<double> nb(0.0, 0.02), nd(0.0, 0.05);
  std::uniform_real_distribution<double> u(0.0, 1.0);
  const int sizes[][2] = {{1500, 1400}, {1800, 1650}, {2300, 2100}, {40, 35}, {700, 4}, {5, 600}, {0, 7}, {9, 0}};
  for (const auto& sz : sizes) {
    const int m = sz[0], k = sz[1];
    const bool dense = m >= 1000;
    std::vector<double> pb(m), pd(m), qb(k), qd(k);
    for (int i = 0; i < m; ++i) {
      pb[i] = float(dense ? nb(g) : u(g));
      pd[i] = float(pb[i] + (dense ? std::fabs(nd(g)) : 0.3 * u(g)));
    }
    for (int j = 0; j < k; ++j) {
      qb[j] = float(dense ? nb(g) : u(g));
      qd[j] = float(qb[j] + (dense ? std::fabs(nd(g)) : 0.3 * u(g)));
    }
    std::vector<int32_t> match(m > 0 ? m : 1);
    double cost = 0, cost2 = 0;
    int rc = ts_assign(m, pb.data(), pd.data(), k, qb.data(), qd.data(), match.data(), &cost);
    if (rc != 0) {
      std::printf("ts_assign %d x %d: rc %d\n", m, k, rc);
      return 1;
    }
    rc = ts_assign_auction(m, pb.data(), pd.data(), k, qb.data(), qd.data(), 0.01, match.data(),
                           &cost2);
    if (rc != 0 || cost2 < cost * (1 - 1e-12)) {
      std::printf("ts_assign_auction %d x %d: rc %d cost %.17g < %.17g\n", m, k, rc, cost2, cost);
      return 1;
    }
    std::printf("%d x %d: cost %.12g (precision 0.01: %.12g)\n", m, k, cost, cost2);
  }
  return 0;
}
