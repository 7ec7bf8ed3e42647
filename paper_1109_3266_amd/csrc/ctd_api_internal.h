// Host-side object layouts behind the opaque C handles, and runtime helpers
// shared by the C-ABI translation units (ctd_api.cpp, ctd_server.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <string>
#include <vector>

#include "ctd.h"
#include "ctd_internal.h"

namespace ctd {

constexpr int kSigmaBlocks = 1024;

struct RoundItem {
  const CaseDev *cd;
  uint64_t h_begin, n;
  std::vector<unsigned long long> prefix;
  const int32_t *beamlets = nullptr;   // Alg. A1 beamlets of the round, or null
  int step_kind = 0;                   // kStepPlain, kStepDeferred or kStepMacro
  int tab_n = 0, tab_ne = 0;           // the case's mu/rho rows and energy nodes
};

}  // namespace ctd

struct ctd_ctx {
  int device = 0;
  hipStream_t own = nullptr;
  hipStream_t stream = nullptr;
  int n_cu = 0;
  std::string err;
  struct Slot {
    void *host = nullptr;
    void *dev = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
  };
  std::vector<Slot> slots;  // staging ring for per-round launch tables
  size_t next_slot = 0;
  double *sigma_scratch = nullptr;
  double *sigma_host = nullptr;
  unsigned int *pack_stats = nullptr;  // [kPackStats] phantom statistics of k_pack
  bool xcd_tally_ok = false;  // every XCC id < kTallyCopies
  unsigned int max_xcc = 0;
  int lds_per_cu = 160 * 1024, lds_per_block = 64 * 1024;  // device LDS limits
  // device address of this device's static round table (ctd_run_batches_static),
  // looked up at creation with the device current; null if the lookup failed
  void *static_table = nullptr;
  // ctd_debug_fail_next_round: the next round fails after its first launch
  bool fail_next_round = false;
};

struct ctd_phantom {
  int device = 0;         // device holding the arrays
  ctd_grid g{};
  int64_t V = 0;
  uint2 *vox = nullptr;   // packed (rho bits, material) records
  uint8_t *vox8 = nullptr;  // palette indices when npal > 0
  uint2 *palette = nullptr; // [256] distinct records when npal > 0
  int npal = 0;
  // bound grids (8-byte record layout): block classes for blocks of 1, 2, 4
  // voxels per edge, the class table [256] (density level bits, material)
  // and each material's (first class, level count)
  uint8_t *bgrid[3] = {nullptr, nullptr, nullptr};
  uint2 *bclass = nullptr;
  int2 *bclass_range = nullptr;
  int nclass = 0;
  std::vector<uint2> bclass_host;   // host copy of the class table
  double rho_max[256] = {};
  double rho_min[256] = {};
  bool present[256] = {};
  uint32_t count[256] = {};   // voxels of each material
  int max_mat = 0;
  std::atomic<int> refs{0};
};

struct ctd_matset {
  int device = 0;         // device holding the tables
  ctd_egrid eg{};
  int M = 0, ncomp = 1, nzc = 0, nzr = 0;
  std::vector<float> mu_rho;  // host copy [M][ne][3]
  float4 *d_mu = nullptr;
  float4 *d_comp = nullptr;
  float4 *d_rayl = nullptr;
  std::atomic<int> refs{0};
};

struct ctd_spectrum {
  std::vector<double> lo, w;
  double width = 0.0;
  std::atomic<int> refs{0};
};

struct ctd_geometry {
  ctd_geom g{};
  std::vector<float4> proj_sc;   // per projection (sin phi, cos phi, z offset, 0)
  std::vector<double> fl_cdf;    // fluence map running sums C_I (empty: uniform field)
  std::vector<int32_t> fl_guide; // [2^fl_gbits] first beamlet with C_I > k F / 2^gbits
  int32_t fl_gbits = 0;
  std::vector<float> fl_f;       // map intensities, kept for Alg. A1 chains
  std::atomic<int> refs{0};
};

struct ctd_case {
  ctd_ctx *ctx = nullptr;
  ctd_phantom *ph = nullptr;
  ctd_matset *ms = nullptr;
  ctd_spectrum *sp = nullptr;
  ctd_geometry *geo = nullptr;
  ctd_params p{};
  double e_max = 0.0;
  ctd_tuning tune{};
  std::vector<float> mu_max;
  ctd::CaseDev desc{};
  ctd::CaseDev *d_desc = nullptr;
  float *d_mu_max = nullptr;
  float *d_bin_lo = nullptr;
  float4 *d_proj = nullptr;
  double *d_fl_cdf = nullptr;
  int32_t *d_fl_guide = nullptr;
  float *d_fl_f = nullptr;         // Alg. A1: intensities [N_f]
  int32_t *d_mh_state = nullptr;   // Alg. A1: last beamlet of each chain [C]
  int32_t *d_mh_beam = nullptr;    // Alg. A1: beamlets of the current round
  uint64_t mh_cap = 0;
  float *d_mc_f = nullptr;         // MACRO tracking: majorant factors [n_band][cells]
  float *d_bnd = nullptr;          // bound-test sums per material and energy cell
  bool use_bound_grid = false;     // the phantom's bound grid serves this case
  int mc_cs = 0, mc_n[3] = {0, 0, 0}, mc_classes = 0, mc_shift = 0, mc_bands = 0;
  unsigned long long *d_tally = nullptr;
  int tally_copies = 1;     // 1, or kTallyCopies once tally_mode 1 is selected
  long long *d_s1 = nullptr;
  unsigned long long *d_s2 = nullptr;
  unsigned long long *d_acc = nullptr;
  ctd_event *d_log = nullptr;
  unsigned long long *d_log_n = nullptr;
  uint64_t log_h0 = 0, log_h1 = 0, log_cap = 0;
  uint64_t h_next = 0;      // next history id
  uint32_t batches = 0;     // batches folded
  // smallest and largest batch folded so far: the batch statistics need
  // batches of equal size (ctd_run's remainder makes some one larger)
  uint64_t batch_min = UINT64_MAX, batch_max = 0;
  struct Timing {
    hipEvent_t a, b, c;
  };
  std::vector<Timing> timing;
  double transport_ms = 0.0, fold_ms = 0.0;
  double sigma_local = NAN, sigma_paper = NAN;
  double s1_bound = 0.0, s2_bound = 0.0;  // upper bounds on any voxel's S1, S2
  bool in_server = false;
  // a run call failed after enqueueing part of its work: the sums, counters
  // and history ids are undefined until ctd_case_reset
  bool failed = false;
};

namespace ctd {

int set_err(ctd_ctx *ctx, int code, const char *fmt, ...);
int hip_err(ctd_ctx *ctx, hipError_t e, const char *what);
int upload_desc(ctd_ctx *ctx, ctd_case *cs);
void fill_desc(ctd_case *cs);
void free_case_buffers(ctd_case *cs);
// One transport launch over items, which share one step kind.
int submit_round(ctd_ctx *ctx, const std::vector<RoundItem> &items, const ctd_tuning &t,
                 bool with_log);
ctd_tuning default_tuning(const ctd_ctx *ctx);
// The step a case's histories take under tuning t (kStep*).
int step_kind(const ctd_case *cs, const ctd_tuning &t);
int batch_prefix(ctd_ctx *ctx, const ctd_case *cs, uint64_t n,
                 std::vector<unsigned long long> &prefix);
int run_round(ctd_ctx *ctx, std::vector<ctd_case *> &cases, const std::vector<uint64_t> &n,
              const ctd_tuning &t);
std::vector<uint64_t> split_batches(uint64_t n, int nb);
int sigma_now(ctd_ctx *ctx, ctd_case *cs, int kind, double frac, double *out);
// Enqueue the sigma-bar reduction of a case on ctx->stream and the copy of
// its three results (sigma-bar, D_max, voxels counted) to host_out, which
// should be pinned; nothing waits.
int sigma_async(ctd_ctx *ctx, ctd_case *cs, int kind, double frac, double *host_out);
// CTD_OK when the case's folded batches, together with `next` more of
// next_size histories (none when next_size = 0), differ in size by at most
// one history; else CTD_EINVAL with a message.
int check_batch_sizes(ctd_ctx *ctx, const ctd_case *cs, uint64_t next_size);
int run_batches(ctd_ctx *ctx, ctd_case *cs, uint64_t batch, uint64_t count);
// Run-to-sigma schedule shared by ctd_run_to_sigma and the server: batches to
// add after `have` batches at sigma-bar `sig` (0 = stop).
uint64_t sigma_plan(uint64_t have, double sig, double target, uint64_t max_batches);
int ensure_tally_copies(ctd_ctx *ctx, ctd_case *cs, int copies);
// Device bytes a case over V voxels allocates (batch tally copies, S1/S2
// sums, counters, projection and fluence tables, Alg. A1 buffers for rounds
// of up to round_histories).
uint64_t case_footprint(const ctd_grid &g, const ctd_geometry *geo, const ctd_params &p,
                        int ne, int tally_copies, uint64_t round_histories);
// Alg. A1 beamlet buffer of at least n entries.
int ensure_mh_buffer(ctd_ctx *ctx, ctd_case *cs, uint64_t n);
// MACRO tracking (ctd_macro.cpp): cells per axis for edge cs (returns the
// cell count) and the per-band, per-cell majorant factors of a case.
int macro_edge(const ctd_grid &g, int requested);
int macro_cells(const ctd_grid &g, int cs, int n[3]);
int build_macro(ctd_ctx *ctx, ctd_case *cs);
// The tracking mode CTD_TRACK_AUTO resolves to for these inputs.
int auto_tracking(const ctd_phantom *ph, const ctd_matset *ms, const ctd_spectrum *sp,
                  bool rayleigh);

}  // namespace ctd
