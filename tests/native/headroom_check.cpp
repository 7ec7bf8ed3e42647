// Drives the fixed-point headroom decision (ctd_headroom.h) through a
// sequence of batches and prints one line per step: verdict, the bounds it
// leaves, and the bounds the caller keeps.  Reads "n e_max max_s1 max_s2_hi"
// lines from stdin; the recorded maxima are used only when the first stage
// asks for them, as the library does.
#include <cstdint>
#include <cstdio>

#include "ctd_headroom.h"

int main() {
  double s1b = 0.0, s2b = 0.0;
  double n, e;
  unsigned long long m1, m2;
  while (std::scanf("%lf %lf %llu %llu", &n, &e, &m1, &m2) == 4) {
    double s1 = 0.0, s2 = 0.0;
    int v = ctd::headroom_bounds(n, e, s1b, s2b, &s1, &s2);
    int w = -1;
    if (v == ctd::kHeadroomNeedExact) w = ctd::headroom_exact(n, e, m1, m2, &s1, &s2);
    const bool ok = v == ctd::kHeadroomOk || w == ctd::kHeadroomOk;
    if (ok) {
      s1b = s1;
      s2b = s2;
    }
    std::printf("%d %d %.17g %.17g\n", v, w, s1b, s2b);
  }
  return 0;
}
