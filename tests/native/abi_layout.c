/* Prints size and field offsets of every struct in include/ctd.h, as the C
 * compiler lays them out, for comparison with the ctypes mirrors. */
#include <stddef.h>
#include <stdio.h>

#include "ctd.h"

#define S(T) printf("%s size %zu\n", #T, sizeof(T));
#define F(T, f) printf("%s.%s %zu\n", #T, #f, offsetof(T, f));

int main(void) {
  S(ctd_grid) F(ctd_grid, dx) F(ctd_grid, origin)
  S(ctd_egrid) F(ctd_egrid, ne)
  S(ctd_geom) F(ctd_geom, src) F(ctd_geom, sad) F(ctd_geom, a0) F(ctd_geom, phi0_deg)
  F(ctd_geom, z_feed) F(ctd_geom, fluence_na) F(ctd_geom, fluence) F(ctd_geom, fluence_chains)
  S(ctd_params) F(ctd_params, seed) F(ctd_params, n_batches) F(ctd_params, sigma_rho_min)
  F(ctd_params, tracking) F(ctd_params, macro_cell)
  S(ctd_balance) F(ctd_balance, q_incident_hi) F(ctd_balance, n_cutoff)
  S(ctd_stats) F(ctd_stats, n_steps) F(ctd_stats, transport_ms) F(ctd_stats, n_batches)
  F(ctd_stats, n_histories) F(ctd_stats, n_crossings) F(ctd_stats, tracking) F(ctd_stats, max_s1)
  F(ctd_stats, max_s2_hi)
  S(ctd_tuning) F(ctd_tuning, tally_mode) F(ctd_tuning, bound_block) F(ctd_tuning, defer_min)
  S(ctd_event) F(ctd_event, vox) F(ctd_event, e) F(ctd_event, E)
  S(ctd_gamma_params) F(ctd_gamma_params, gamma_cap) F(ctd_gamma_params, substeps)
  S(ctd_server_config) F(ctd_server_config, dose_frac) F(ctd_server_config, tuning)
  S(ctd_request_info) F(ctd_request_info, sigma) F(ctd_request_info, t_done)
  S(ctd_server_stats) F(ctd_server_stats, resident_bytes) F(ctd_server_stats, active)
  return 0;
}
