// Host-sanitizer driver of the CPU oracle: diagram, full reduction, assignment
// step and a short solve on small random fields, built with AddressSanitizer
// and UndefinedBehaviorSanitizer.
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

#include "tso.h"

int main() {
  std::mt19937_64 g(3);
  std::uniform_real_distribution<float> u(0.0f, 1.0f);
  const int64_t grids[][3] = {{2, 2, 2}, {5, 4, 3}, {9, 7, 6}, {12, 11, 10}};
  for (const auto& d : grids) {
    const int64_t n = d[0] * d[1] * d[2];
    std::vector<float> f(n);
    for (auto& x : f) x = u(g);
    std::vector<tso_pair> D(8 * n + 16);
    int64_t nd = 0;
    if (tso_diagram(f.data(), d, D.data(), int64_t(D.size()), &nd) != 0) return 1;
    if (n <= 64) {
      std::vector<tso_pair> P(64 * n);
      int64_t np = 0;
      if (tso_pairs(f.data(), d, 1, P.data(), int64_t(P.size()), &np) != 0) return 1;
    }
    tso_signal sig{};
    sig.threshold_rel = 0.1f;
    sig.nonsignal_dim_mask = 7u;
    tso_options opt{0.5f, 0.5f, 20, 0, 1e-6f, 0.01f};
    std::vector<float> out(n);
    tso_report rep{};
    std::vector<double> trace(21);
    if (tso_simplify(f.data(), d, &sig, &opt, out.data(), &rep, trace.data(), 21) < 0) return 1;
    // one assignment step against the diagram itself (every point still)
    std::vector<int32_t> phi(nd, -1), out_phi(nd);
    int64_t ns = 0, nr = 0;
    for (int64_t i = 0; i < nd; ++i)
      if (D[i].essential) phi[i] = int32_t(i);
    if (tso_assign_step(D.data(), nd, phi.data(), D.data(), nd, D.data(), nd, out_phi.data(),
                        &ns, &nr) != 0)
      return 1;
    std::printf("%lldx%lldx%lld: %lld points, %d iterations, %lld still\n", (long long)d[0],
                (long long)d[1], (long long)d[2], (long long)nd, rep.iterations, (long long)ns);
  }
  return 0;
}
