// Bound-test sums of the bound grid (host side, plain C++): for material m
// and energy cell j ([E_j, E_j+1]) a float at or above the interaction sum
// (photoelectric + Compton, + Rayleigh when on) that the Woodcock selection
// forms in float32 anywhere in the cell, so that a block's density level
// times it, rounded, bounds the selection at every density of the block.
//
// The sum over the processes of the largest value the column's linear
// interpolation takes in the cell, rounded up to float with a relative
// margin of 2^-20.  Inside the grid the interpolation weight w = f - j lies
// in [0, 1) exactly, and the float interpolation fma(w, x1 - x0, x0) stays
// within (1 + u)^2 of the larger node (u = 2^-24); the selection's products
// and sums of the non-negative rho-scaled terms add at most (1 + u)^3, and
// 2^-20 = 16u covers both and the final rounding.  In the top cell (E up to
// the last node) the rounding of f = (E - e0) / dE can put w past 1 by about
// 3u (ne - 1); there the column is extended to w = 1 + 4u ne.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstddef>

namespace ctd {

inline float round_up_float(double x) {
  float f = (float)x;
  if ((double)f < x) f = std::nextafter(f, INFINITY);
  return f;
}

// mu_rho [M][ne][3] (pe, Compton, Rayleigh) cm^2/g; out [M][ne - 1].
inline void bound_sums(const float *mu_rho, int M, int ne, bool rayleigh, float *out) {
  const double w_top = 1.0 + 4.0 * 0x1p-24 * ne;
  for (int m = 0; m < M; ++m) {
    const float *r = mu_rho + (size_t)m * ne * 3;
    for (int j = 0; j + 1 < ne; ++j) {
      const float *x0 = r + (size_t)j * 3, *x1 = x0 + 3;
      const double w = j + 2 == ne ? w_top : 1.0;
      auto peak = [&](int k) {   // largest value of the column over the cell
        return std::max((double)x0[k], (double)x0[k] + w * ((double)x1[k] - (double)x0[k]));
      };
      double sum = peak(0) + peak(1);
      if (rayleigh) sum += peak(2);
      out[(size_t)m * (ne - 1) + j] = round_up_float(sum * (1.0 + 0x1p-20));
    }
  }
}

}  // namespace ctd
