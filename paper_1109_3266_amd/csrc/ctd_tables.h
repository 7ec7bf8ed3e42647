// Host FP64 table construction (see ctd_tables.cpp).
#pragma once

#include <cstdint>

namespace ctd {

int build_surface_fp64(int n_e, int n_mu, const double *pdf, int n_zeta, float *out);
float round_up_to_float(double x);
void majorant_fp64(int ne, int M, const float *mu_rho, const double *rho_max, const bool *present,
                   bool rayleigh, float *out);
int alloc_bins(uint64_t n, int nbins, const double *w, uint64_t *counts);

}  // namespace ctd
