// The bound-test sums of ctd_bound.h against the float32 selection they
// bound, evaluated as the transport evaluates it: random tables (steep
// columns, jumps like absorption edges, zero columns), energies anywhere in
// the grid including the nodes and the top, the energy-cell weight formed
// from (E - e0) * (1/dE) in float, columns interpolated with fma, and the
// selection sum rho a + rho b (+ rho c) at the block's level and at lower
// densities.  Prints "ok <checks> <largest selection/bound ratio>" or the
// first violation.  Arguments: seed trials.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "ctd_bound.h"

namespace {

struct Rng {
  uint64_t s;
  double u() {   // [0, 1)
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(s >> 11) * 0x1p-53;
  }
};

}  // namespace

int main(int argc, char **argv) {
  Rng g{argc > 1 ? std::strtoull(argv[1], nullptr, 10) : 1ull};
  const int trials = argc > 2 ? std::atoi(argv[2]) : 200;
  long checks = 0;
  double worst = 0.0;
  for (int t = 0; t < trials; ++t) {
    const int M = 1 + (int)(g.u() * 6), ne = 3 + (int)(g.u() * 300);
    const float e0 = (float)(1.0 + g.u() * 4.0), de = (float)(0.25 + g.u() * 2.0);
    const bool rayleigh = g.u() < 0.5;
    std::vector<float> tab((size_t)M * ne * 3);
    for (int m = 0; m < M; ++m)
      for (int k = 0; k < 3; ++k) {
        double v = std::pow(10.0, -3.0 + 4.0 * g.u());
        const bool zero = g.u() < 0.1;
        for (int j = 0; j < ne; ++j) {
          v *= std::exp((g.u() - 0.6) * 0.3);          // smooth drift
          if (g.u() < 0.02) v *= 1.0 + 9.0 * g.u();    // an edge
          tab[((size_t)m * ne + j) * 3 + k] = zero ? 0.0f : (float)v;
        }
      }
    std::vector<float> bnd((size_t)M * (ne - 1));
    ctd::bound_sums(tab.data(), M, ne, rayleigh, bnd.data());
    const float inv_de = (float)(1.0 / (double)de);
    const double etop = (double)e0 + (double)(ne - 1) * (double)de;
    for (int q = 0; q < 400; ++q) {
      double Ed;
      const double r = g.u();
      if (r < 0.1) Ed = etop;                                   // the top node
      else if (r < 0.3) Ed = (double)e0 + (int)(g.u() * (ne - 1)) * (double)de;   // a node
      else Ed = (double)e0 + g.u() * (etop - (double)e0);
      float E = (float)Ed;
      if ((double)E > etop) E = std::nextafter(E, 0.0f);       // sampled energies stay below
      if (E < e0) E = e0;
      const float f = (E - e0) * inv_de;
      const int j = std::min(std::max((int)f, 0), ne - 2);
      const float w = f - (float)j;
      for (int m = 0; m < M; ++m) {
        const float *x0 = &tab[((size_t)m * ne + j) * 3], *x1 = x0 + 3;
        const float a = std::fmaf(w, x1[0] - x0[0], x0[0]);
        const float b = std::fmaf(w, x1[1] - x0[1], x0[1]);
        const float c = rayleigh ? std::fmaf(w, x1[2] - x0[2], x0[2]) : 0.0f;
        const float rho_c = (float)std::pow(10.0, -3.0 + 3.5 * g.u());
        const float B = rho_c * bnd[(size_t)m * (ne - 1) + j];
        for (int s = 0; s < 3; ++s) {
          const float rho = s == 0 ? rho_c : rho_c * (float)g.u();
          float sum = rho * a + rho * b;
          if (rayleigh) sum = sum + rho * c;
          ++checks;
          if (!(B >= sum)) {
            std::printf("violation: trial %d m %d j %d w %.9g rho %.9g bound %.9g sum %.9g\n", t, m,
                        j, (double)w, (double)rho, (double)B, (double)sum);
            return 0;
          }
          if (B > 0.0f) worst = std::max(worst, (double)sum / (double)B);
        }
      }
    }
  }
  std::printf("ok %ld %.9f\n", checks, worst);
  return 0;
}
