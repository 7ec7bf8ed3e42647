// Host-side FP64 table construction for the transport library:
//  - inverse-CDF surfaces (Jia et al., Sec. 2.2.2: pdf at equally spaced mu,
//    numerical cumulative distribution, inverse at equally spaced zeta);
//  - the Woodcock majorant mu_max(E) (Sec. 2.1);
//  - the per-batch split of histories over 1 keV spectrum bins (Sec. 2.2.5).
#include <cmath>
#include <cstdint>
#include <vector>

#include "ctd.h"
#include "ctd_tables.h"

namespace ctd {

int build_surface_fp64(int n_e, int n_mu, const double *pdf, int n_zeta, float *out) {
  if (n_e < 1 || n_mu < 2 || n_zeta < 2 || !pdf || !out) return CTD_EINVAL;
  const double h = 2.0 / (double)(n_mu - 1);
  std::vector<double> P((size_t)n_mu), mu((size_t)n_mu);
  for (int k = 0; k < n_mu; ++k) mu[k] = -1.0 + 2.0 * (double)k / (double)(n_mu - 1);
  for (int j = 0; j < n_e; ++j) {
    const double *p = pdf + (size_t)j * n_mu;
    for (int k = 0; k < n_mu; ++k)
      if (!(p[k] >= 0.0) || !std::isfinite(p[k])) return CTD_EINVAL;
    // trapezoid rule, accumulated in order
    P[0] = 0.0;
    for (int k = 1; k < n_mu; ++k) P[k] = P[k - 1] + 0.5 * (p[k - 1] + p[k]) * h;
    const double Z = P[n_mu - 1];
    if (!(Z > 0.0)) return CTD_EINVAL;
    for (int k = 0; k < n_mu; ++k) P[k] = P[k] / Z;
    // invert at zeta_i: largest k <= n_mu - 2 with P_k <= zeta, linear between nodes
    int k = 0;
    for (int i = 0; i < n_zeta; ++i) {
      const double z = (double)i / (double)(n_zeta - 1);
      while (k + 1 <= n_mu - 2 && P[k + 1] <= z) ++k;
      const double den = P[k + 1] - P[k];
      const double m = den > 0.0 ? mu[k] + h * (z - P[k]) / den : mu[k];
      out[(size_t)j * n_zeta + i] = (float)m;
    }
  }
  return CTD_OK;
}

float round_up_to_float(double x) {
  float f = (float)x;
  if ((double)f < x) f = std::nextafter(f, INFINITY);
  return f;
}

void majorant_fp64(int ne, int M, const float *mu_rho, const double *rho_max, const bool *present,
                   bool rayleigh, float *out) {
  for (int j = 0; j < ne; ++j) {
    double best = 0.0;
    for (int m = 0; m < M; ++m) {
      if (!present[m]) continue;
      const float *t = mu_rho + ((size_t)m * ne + j) * 3;
      double s = (double)t[0] + (double)t[1];
      if (rayleigh) s += (double)t[2];
      const double v = rho_max[m] * s;
      if (v > best) best = v;
    }
    out[j] = round_up_to_float(best * (1.0 + 1.0 / 1048576.0));
  }
}

int alloc_bins(uint64_t n, int nbins, const double *w, uint64_t *counts) {
  double W = 0.0;
  for (int j = 0; j < nbins; ++j) {
    if (!(w[j] >= 0.0)) return CTD_EINVAL;
    W += w[j];
  }
  if (!(W > 0.0)) return CTD_EINVAL;
  // bin j's share n w_j / W, recomputed by the same operations wherever it is
  // needed (no scratch arrays: the static-table entry point allocates nothing)
  auto share = [&](int j) { return ((double)n * w[j]) / W; };
  uint64_t used = 0;
  for (int j = 0; j < nbins; ++j) {
    counts[j] = (uint64_t)std::floor(share(j));
    used += counts[j];
  }
  if (used > n) return CTD_EINVAL;
  uint64_t rem = n - used;
  if (rem > (uint64_t)nbins) return CTD_EINVAL;
  // the rem largest fractional parts get one more (ties: lower bin first); a
  // bin already given one has a count above the floor of its share
  for (uint64_t r = 0; r < rem; ++r) {
    int best = -1;
    double best_f = 0.0;
    for (int j = 0; j < nbins; ++j) {
      const double q = share(j), fl = std::floor(q);
      if (counts[j] != (uint64_t)fl) continue;
      if (best < 0 || q - fl > best_f) {
        best = j;
        best_f = q - fl;
      }
    }
    counts[best] += 1;
  }
  return CTD_OK;
}

}  // namespace ctd

extern "C" int32_t ctd_surface_build(int32_t n_e, int32_t n_mu, const double *pdf, int32_t n_zeta,
                                     float *out) {
  return ctd::build_surface_fp64(n_e, n_mu, pdf, n_zeta, out);
}
